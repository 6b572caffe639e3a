"""Build step for the gfx950 library: compiles csrc/*.hip with hipcc into
libdebyefit.so next to this file (in-tree, so the GPU machine loads exactly the
library built here)."""
import concurrent.futures as cf
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "csrc")
INC = os.path.join(os.path.dirname(_HERE), "include")
LIB = os.path.join(_HERE, "libdebyefit.so")
ARCH = os.environ.get("DEBYEFIT_ARCH", "gfx950")

COMMON = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", f"-I{INC}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
# per-file extra flags: the optimiser updates must be rounded operation by operation
EXTRA = {"pso.hip": ["-ffp-contract=off"], "de.hip": ["-ffp-contract=off"], "da.hip": ["-ffp-contract=off"]}
SOURCES = ["fit_ragged.hip", "fit_eval.hip", "fit_grad.hip", "fit_dd.hip", "material.hip", "pso.hip", "de.hip", "da.hip", "lbfgs.hip", "api.hip", "auto.hip",
           "noalloc.hip"]


def _compile(name, objdir, verbose):
    src = os.path.join(SRC, name)
    obj = os.path.join(objdir, name + ".o")
    cmd = COMMON + EXTRA.get(name, []) + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{r.stderr}")
    return obj


def build(verbose=False, jobs=None):
    objdir = os.path.join(_HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda n: _compile(n, objdir, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
