"""The gprMax front end end to end on the GPU: Listing 1 and the other
layouts are fitted in one run, the reported errors equal the oracle's error
of the returned expansions, and the written commands parse back to them."""
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2109_01928_amd import gprmax as G

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(__file__)


def _targets(orc, c, n_freq=G.N_FREQ):
    if c.table is not None:
        f, er, ei = c.table
        return 2 * np.pi * f, er, ei
    om = 2 * np.pi * np.geomspace(c.f_lo, c.f_hi, n_freq)
    er, ei = orc.material_eval([c.kind], c.params[None], [0, len(om)], om)
    return om, er, ei


def test_translate_end_to_end(orc, tmp_path):
    listing1 = [l for l in open(os.path.join(HERE, "golden", "gprmax_listings.txt")) if l.startswith("#hav")][0]
    f = np.geomspace(1e7, 1e10, 60)
    x = 2 * np.pi * f * 3e-10
    np.savetxt(tmp_path / "wet.txt", np.stack([f, 5 + 20 / (1 + x * x), 20 * x / (1 + x * x)], 1))
    text = (listing1 +
            "#jonscher: 1e6 1e10 0.4 5.0 10.0 1e8 0.01 1 0 6 concrete 7\n"
            "#crim: 1e6 1e10 0.5 0.2 4.9 75 9.2e-12 6.0 0 1 0 -1 soil\n"
            "#raw_data: wet.txt 0 1 0 2 wet\n")
    cmds = G.parse(text, str(tmp_path))
    res = G.fit(cmds, particles=48, iters=60, polish_steps=20)
    for c, (einf, d_eps, tau, err) in zip(cmds, res):
        om, er, ei = _targets(orc, c)
        ref = orc.afe(om, er, ei, d_eps, tau, einf)
        print(f"{c.command} {c.ident}: {len(d_eps)} poles, AFE GPU {err:.6f} % oracle {ref:.6f} %")
        assert err == pytest.approx(ref, rel=1e-9)
        assert np.all(d_eps >= 0)                       # flipped weights
        lb, ub = G.tau_bounds(c.f_lo, c.f_hi)
        assert np.all((np.log10(tau) >= lb - 1e-12) & (np.log10(tau) <= ub + 1e-12))
    # Listing 1 with five poles: a useful fit (the paper reports 8.48 % for PSO-DLS)
    assert len(res[0][1]) == 5 and res[0][3] < 10.0
    assert res[2][3] < 5.0 or len(res[2][1]) == G.MAX_AUTO_POLES
    assert len(res[3][1]) == 2 and res[3][3] < 1e-3       # a one-term Debye table: two poles fit it exactly
    out = G.translate(text, str(tmp_path), particles=48, iters=60, polish_steps=20)
    mats = re.findall(r"^#material: (\S+) (\S+) (\S+) (\S+) (\S+)$", out, re.M)
    disp = re.findall(r"^#add_dispersion_debye: (\d+) (.*) (\S+)$", out, re.M)
    assert [m[4] for m in mats] == ["Kelley", "concrete", "soil", "wet"]
    assert mats[0][1:4] == ("0.1", "1", "0")
    for (n, pairs, ident), (einf, d_eps, tau, err) in zip(disp, res):
        vals = np.array(pairs.split(), float)
        assert int(n) == len(d_eps) == len(vals) // 2
        np.testing.assert_allclose(vals[0::2], d_eps, rtol=1e-4, atol=1e-4)
        np.testing.assert_allclose(vals[1::2], tau, rtol=1e-4)
