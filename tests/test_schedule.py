"""CPU checks of the work schedule a plan builds for one pole-count bucket
(debye_schedule_preview, host only): every candidate sits in exactly one wave
slot with its own material, padding only closes an XCD's last tile, the
estimated work per XCD is balanced, and the uniform-tile form (one material
per wave, at any split) is detected exactly when it holds."""
import numpy as np
import pytest

import paper_2109_01928_amd as D


def _offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def _tile_time(F, SF, N):
    return -(-F // SF) + 0.05 * N * N


def _check_cover(lc, lm, xo, cand_off, mats, cpw):
    n_tiles = len(lc) // cpw
    assert len(lc) == n_tiles * cpw and xo[0] == 0 and xo[8] == n_tiles
    assert np.all(np.diff(xo) >= 0)
    want = np.concatenate([np.arange(cand_off[m], cand_off[m + 1]) for m in mats]) if len(mats) else np.zeros(0)
    real = lc[lc >= 0]
    assert np.array_equal(np.sort(real), np.sort(want))  # each candidate exactly once
    mat_of = np.searchsorted(cand_off, real, side="right") - 1
    assert np.array_equal(lm[lc >= 0], mat_of)
    # padding (-1) only at the end of an XCD's last tile
    for x in range(8):
        seg = lc[xo[x] * cpw:xo[x + 1] * cpw]
        pad = np.flatnonzero(seg < 0)
        if len(pad):
            assert pad[0] >= len(seg) - cpw + 1 and np.all(seg[pad[0]:] < 0)


def _xcd_loads(lc, lm, xo, f_off, cpw, SF, N):
    loads = np.zeros(8)
    for x in range(8):
        for t in range(xo[x], xo[x + 1]):
            lane = slice(t * cpw, (t + 1) * cpw)
            ms = lm[lane][lc[lane] >= 0]
            loads[x] += max(_tile_time(f_off[m + 1] - f_off[m], SF, N) for m in set(ms.tolist()))
    return loads


def test_uniform_swarms_fill_whole_waves():
    M, P, F, N = 1024, 256, 1000, 8
    f_off, cand_off = _offsets([F] * M), _offsets([P] * M)
    mats = np.arange(M)
    lc, lm, xo, uni = D.schedule_preview(f_off, cand_off, mats, N, 1, 1)
    _check_cover(lc, lm, xo, cand_off, mats, 64)
    assert uni and len(lc) == M * P
    assert np.all(np.diff(xo) == M * P // 64 // 8)
    # a material's candidates stay on one XCD (its spectrum in one L2)
    for x in range(8):
        ms = set(lm[xo[x] * 64:xo[x + 1] * 64].tolist())
        for y in range(x + 1, 8):
            assert not ms & set(lm[xo[y] * 64:xo[y + 1] * 64].tolist())


@pytest.mark.parametrize("N,SP,SF", [(4, 1, 1), (8, 1, 2), (12, 2, 2), (20, 4, 4), (6, 1, 8)])
def test_ragged_batch_is_covered_and_balanced(N, SP, SF):
    rng = np.random.default_rng(7 + N)
    M = 300
    P = rng.integers(1, 400, M)
    F = rng.integers(20, 3000, M)
    f_off, cand_off = _offsets(F), _offsets(P)
    mats = np.sort(rng.choice(M, 200, replace=False)).astype(np.int32)
    cpw = 64 // (SP * SF)
    lc, lm, xo, uni = D.schedule_preview(f_off, cand_off, mats, N, SP, SF)
    _check_cover(lc, lm, xo, cand_off, mats, cpw)
    assert not uni
    loads = _xcd_loads(lc, lm, xo, f_off, cpw, SF, N)
    assert loads.max() / loads.mean() < 1.05, loads


def test_one_large_material_spreads_over_every_xcd():
    # a single swarm of 64k candidates is cut into pieces for all 8 XCDs
    f_off, cand_off = _offsets([500]), _offsets([65536])
    lc, lm, xo, uni = D.schedule_preview(f_off, cand_off, [0], 8, 1, 1)
    _check_cover(lc, lm, xo, cand_off, [0], 64)
    assert uni and np.all(np.diff(xo) == 128)


def test_uniform_detection():
    f_off = _offsets([100] * 4)
    # 128 candidates per material: whole waves of one material at split 1
    assert D.schedule_preview(f_off, _offsets([128] * 4), range(4), 5, 1, 1)[3]
    # 4 x 100: one material per XCD, each padded to whole waves
    assert D.schedule_preview(f_off, _offsets([100] * 4), range(4), 5, 1, 1)[3]
    # 16 x 100: an XCD packs several materials and some waves hold two
    lc, lm, xo, uni = D.schedule_preview(_offsets([100] * 16), _offsets([100] * 16), range(16), 5, 1, 1)
    assert not uni
    assert any(len(set(lm[t * 64:(t + 1) * 64][lc[t * 64:(t + 1) * 64] >= 0].tolist())) > 1 for t in range(xo[8]))
    # with a frequency or pole split, whole waves of one material too
    assert D.schedule_preview(f_off, _offsets([128] * 4), range(4), 5, 1, 2)[3]
    assert D.schedule_preview(f_off, _offsets([128] * 4), range(4), 12, 2, 1)[3]
    assert D.schedule_preview(f_off, _offsets([48] * 4), range(4), 20, 4, 4)[3]
    # 16 x 12 candidates at 8 per wave: pieces of 4 share waves
    assert not D.schedule_preview(_offsets([100] * 16), _offsets([12] * 16), range(16), 20, 4, 2)[3]
    # one material padded to a whole wave is still uniform
    assert D.schedule_preview(_offsets([100]), _offsets([10]), [0], 5, 1, 1)[3]
    # a spectrum of 2^29 points or more is past the uniform form's 32-bit
    # byte offsets: the general form (64-bit point indices) takes it
    assert D.schedule_preview(_offsets([2**29 - 1]), _offsets([8]), [0], 2, 1, 64)[3]
    assert not D.schedule_preview(_offsets([2**29]), _offsets([8]), [0], 2, 1, 64)[3]
    assert not D.schedule_preview(_offsets([100, 2**29 + 5]), _offsets([64, 64]), [0, 1], 2, 1, 1)[3]


def test_empty_bucket_and_bad_arguments():
    f_off, cand_off = _offsets([100, 100]), _offsets([0, 0])
    lc, lm, xo, uni = D.schedule_preview(f_off, cand_off, [0, 1], 4, 1, 1)
    assert len(lc) == 0 and np.all(xo == 0)
    for N, SP, SF in [(0, 1, 1), (D.MAX_POLES + 1, 1, 1), (4, 3, 1), (4, 1, 3), (4, 4, 32)]:
        with pytest.raises(D.DebyeError):
            D.schedule_preview(_offsets([10]), _offsets([10]), [0], N, SP, SF)
