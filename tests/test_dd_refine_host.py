"""The double-double routines of the extended-precision refinement
(DEBYE_FLAG_DD_REFINE), checked on the host against 50-digit decimal
arithmetic.

The routines are taken from the kernel source as written (the block from the
double-double pair type to the Debye basis term), compiled for the host with
contraction off (as the kernel compiles them), with an exactly rounded
reciprocal standing in for the hardware one (the kernel's is within half an
ulp, which the routines' correction step absorbs).  Checked: 10^t for t in
[-30, 30] to about 2^-95 (and the exact powers 10^0 ... 10^22 exactly), and
the basis term x / (1 + x^2), x = w tau, to about 2^-100 over the admissible
range of w and tau.  A dropped term (the low part of ln 10, of ln 2 or of the
product's error) or a short Taylor series fails these bounds by many orders of
magnitude.
"""
import ctypes
import os
import shutil
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2109_01928_amd", "csrc", "fit_kernel.hpp")


def _host_source():
    s = open(SRC).read()
    a = s.index("struct ddv {")
    b = s.index("// Debye basis of the owned poles at one frequency")
    block = s[a:s.rindex("// ----", a, b)]
    block = block.replace("__device__ __forceinline__", "static inline").replace("__device__ __noinline__", "static")
    return ("#include <cmath>\n"
            "static inline double rcp_nr(double d) { return 1.0 / d; }\n" + block +
            'extern "C" void exp10_many(int n, const double *t, double *h, double *l) {\n'
            "  for (int i = 0; i < n; ++i) { ddv v = exp10_dd(t[i]); h[i] = v.h; l[i] = v.l; }\n}\n"
            'extern "C" void basis_many(int n, const double *w, const double *th, const double *tl, double *h,'
            " double *l) {\n"
            "  for (int i = 0; i < n; ++i) { ddv v = dd_debye_I(w[i], th[i], tl[i]); h[i] = v.h; l[i] = v.l; }\n}\n")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("ddhost")
    src, so = d / "dd.cpp", d / "libdd.so"
    src.write_text(_host_source())
    subprocess.run([cxx, "-O2", "-ffp-contract=off", "-Wno-unknown-pragmas", "-shared", "-fPIC", "-o", str(so),
                    str(src)], check=True)
    L = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    L.exp10_many.argtypes = [ctypes.c_int, dp, dp, dp]
    L.basis_many.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _exp10(L, t):
    t = np.ascontiguousarray(t, np.float64)
    h, l = np.empty_like(t), np.empty_like(t)
    L.exp10_many(len(t), _p(t), _p(h), _p(l))
    return h, l


def test_exp10_dd_against_decimal(lib):
    getcontext().prec = 50
    rng = np.random.default_rng(5)
    t = np.concatenate([rng.uniform(-30.0, 30.0, 1500), [0.0, 0.5, -0.5, 1e-17, -1e-17, 30.0, -30.0, 17.3, -12.7]])
    h, l = _exp10(lib, t)
    worst = max(abs((Decimal(float(a)) + Decimal(float(b))) / Decimal(10) ** Decimal(float(x)) - 1)
                for x, a, b in zip(t, h, l))
    assert float(worst) < 2.0 ** -90, float(worst)
    # exact powers of ten: exact, with a vanishing low part
    k = np.arange(0, 23, dtype=np.float64)
    h, l = _exp10(lib, k)
    assert np.array_equal(h, 10.0 ** k)
    assert np.all(np.abs(l) <= 2.0 ** -95 * h)


def test_debye_term_against_decimal(lib):
    getcontext().prec = 50
    rng = np.random.default_rng(6)
    n = 3000
    th, tl = _exp10(lib, rng.uniform(-30.0, 30.0, n))
    w = 2.0 * np.pi * 10.0 ** rng.uniform(-3.0, 44.0, n)
    h, l = np.empty(n), np.empty(n)
    lib.basis_many(n, _p(w), _p(th), _p(tl), _p(h), _p(l))
    worst = Decimal(0)
    for i in range(n):
        x = Decimal(float(w[i])) * (Decimal(float(th[i])) + Decimal(float(tl[i])))
        exact = x / (1 + x * x)
        worst = max(worst, abs((Decimal(float(h[i])) + Decimal(float(l[i]))) / exact - 1))
    assert float(worst) < 2.0 ** -98, float(worst)
