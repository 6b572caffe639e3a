"""The gprMax command front end on the CPU: Listing 1 parses into the paper's
fields, Listing 2 is reproduced character for character from its own
numbers, the other command layouts and their errors, and the replacement of
commands in an input file (the fit itself is stubbed here; the GPU test runs it)."""
import os

import numpy as np
import pytest

from paper_2109_01928_amd import gprmax as G

HERE = os.path.dirname(__file__)


def _listings():
    lines = [l.rstrip("\n") for l in open(os.path.join(HERE, "golden", "gprmax_listings.txt")) if l.strip()]
    return lines[1], lines[2], lines[3]


def test_listing1_parses_into_the_papers_fields():
    l1, _, _ = _listings()
    (c,) = G.parse(l1)
    assert c.command == "#havriliak_negami" and c.kind == 1
    assert (c.f_lo, c.f_hi) == (1e7, 1e11)
    np.testing.assert_array_equal(c.params[:5], [2.7, 5.9, 9.4e-10, 0.91, 0.45])   # eps_inf, d_eps, tau0, a, b
    assert (c.sigma, c.mu_r, c.sigma_m, c.n_poles, c.ident, c.seed) == ("0.1", "1", "0", 5, "Kelley", 0)


def test_listing2_reproduced_from_its_numbers():
    l1, l2, l3 = _listings()
    (c,) = G.parse(l1)
    d_eps = [2.3563, 0.6736, 1.1009, 1.2926, 0.3091]
    tau = [4.3677e-10, 1.1623e-11, 1.5180e-9, 9.1048e-11, 1.1131e-12]
    assert G.emit(c, 2.8345, d_eps, tau) == l2 + "\n" + l3 + "\n"


@pytest.mark.parametrize("v,s", [(2.83451, "2.8345"), (0.1, "0.1000"), (1.518e-9, "1.5180e-9"),
                                 (9.10484e-11, "9.1048e-11"), (0.0, "0.0000"), (-3.2e-4, "-3.2000e-4"),
                                 (12.0, "12.0000")])
def test_number_format(v, s):
    assert G.number(v) == s


def test_other_layouts_and_seed(tmp_path):
    text = ("#title: test\n"
            "#jonscher: 1e6 1e10 0.4 5.0 10.0 1e8 0.01 1 0 6 concrete 7\n"
            "#crim: 1e6 1e10 0.5 0.2 4.9 75 9.2e-12 6.0 0 1 0 -1 soil\n")
    table = tmp_path / "tab.txt"
    f = np.geomspace(1e6, 1e9, 30)
    np.savetxt(table, np.stack([f[::-1], 3 + 0 * f, 0.5 + 0 * f], 1), header="f eps' eps''")
    text += f"#raw_data: {table.name} 0 1 0 4 measured\n"
    cmds = G.parse(text, str(tmp_path))
    assert [c.command for c in cmds] == ["#jonscher", "#crim", "#raw_data"]
    j, c, r = cmds
    np.testing.assert_allclose(j.params[:4], [5.0, 10.0, 2 * np.pi * 1e8, 0.4])
    assert j.seed == 7 and j.n_poles == 6
    np.testing.assert_array_equal(c.params[:5], [4.9, 75, 9.2e-12, 0.2, 6.0])
    assert c.n_poles == -1
    assert r.kind == -1 and (r.f_lo, r.f_hi) == (f[0], f[-1]) and np.all(np.diff(r.table[0]) > 0)


@pytest.mark.parametrize("line", [
    "#havriliak_negami: 1e7 1e11 0.91 0.45 2.7 5.9",                       # too few
    "#havriliak_negami: 1e7 1e11 0.91 0.45 2.7 5.9 9.4e-10 0.1 1 0 0 x",   # zero poles
    "#havriliak_negami: 1e11 1e7 0.91 0.45 2.7 5.9 9.4e-10 0.1 1 0 5 x",   # band reversed
    "#crim: 1e6 1e10 0.3 0.2 4.9 75 9.2e-12 6.0 0 1 0 5 soil",             # shape factor
    "#jonscher: 1e6 1e10 0.4 5.0 ten 1e8 0.01 1 0 6 c",                    # not a number
])
def test_malformed_commands_rejected(line):
    with pytest.raises(G.CommandError):
        G.parse(line)


def test_bounds_follow_the_band():
    # the single-HN example's band 1e5 - 1e10 Hz gives the search box [-12, -6]
    assert G.tau_bounds(1e5, 1e10) == (-12.0, -6.0)


def test_translate_replaces_commands_in_place(monkeypatch):
    l1, l2, l3 = _listings()
    monkeypatch.setattr(G, "fit", lambda cmds, **kw: [(2.8345, np.array([2.3563, 0.6736, 1.1009, 1.2926, 0.3091]),
                                                        np.array([4.3677e-10, 1.1623e-11, 1.5180e-9, 9.1048e-11,
                                                                  1.1131e-12]), 8.48)])
    out = G.translate("#domain: 1 1 1\n" + l1 + "\n#dx_dy_dz: 0.1 0.1 0.1\n").splitlines()
    assert out[0] == "#domain: 1 1 1" and out[-1] == "#dx_dy_dz: 0.1 0.1 0.1"
    assert out[1].startswith("Fitted 5 Debye poles (average fractional error 8.48 %)") and not out[1].startswith("#")
    assert out[2] == l2 and out[3] == l3
