"""Pins of the preprocessing oracle (oracle/prep.py), CPU only: hand-worked
values, brute-force loops, conservation laws, and the purpose of the median
step (a static source vanishes, a mover survives)."""

import numpy as np
import pytest

from oracle import prep


def test_median_hand_values():
    f = np.array([1, 5, 3], np.float32).reshape(3, 1, 1)
    out, med = prep.median_subtract(f)
    assert med[0, 0] == 3.0 and list(out[:, 0, 0]) == [-2.0, 2.0, 0.0]
    f = np.array([1, 5, 3, 10], np.float32).reshape(4, 1, 1)
    _, med = prep.median_subtract(f)
    assert med[0, 0] == 4.0
    f = np.array([-2, 7, 7, 7, -9], np.float32).reshape(5, 1, 1)
    assert prep.median_subtract(f)[1][0, 0] == 7.0


def test_median_removes_static_source_keeps_mover():
    n, h, w = 9, 12, 30
    star = np.zeros((h, w))
    star[6, 10] = 50.0
    frames = np.tile(star, (n, 1, 1))
    for i in range(n):  # a mover one pixel per frame along row 3
        frames[i, 3, 5 + 2 * i] += 20.0
    out, med = prep.median_subtract(frames.astype(np.float32))
    assert np.array_equal(med, star)
    assert np.all(out[:, 6, 10] == 0.0)
    for i in range(n):
        assert out[i, 3, 5 + 2 * i] == 20.0
    assert np.count_nonzero(out) == n


def test_coadd_bruteforce_and_times():
    rng = np.random.default_rng(3)
    f = rng.normal(size=(11, 4, 5)).astype(np.float32)
    t = np.cumsum(rng.uniform(0.1, 1, 11))
    out, t_out = prep.coadd(f, 3, t)
    assert out.shape == (3, 4, 5) and t_out.shape == (3,)
    for g in range(3):
        s = np.zeros((4, 5))
        for j in range(3):
            s += f[3 * g + j].astype(np.float64)
        assert np.array_equal(out[g], s)
        assert t_out[g] == pytest.approx((t[3 * g] + t[3 * g + 1] + t[3 * g + 2]) / 3, rel=1e-15)
    c = np.full((6, 2, 2), 1.5, np.float32)
    assert np.all(prep.coadd(c, 6)[0] == 9.0)


def test_bin2x2_bruteforce_and_conservation():
    rng = np.random.default_rng(4)
    f = rng.normal(size=(2, 7, 9)).astype(np.float32)
    b = prep.bin2x2(f)
    assert b.shape == (2, 3, 4)
    for i in range(2):
        for y in range(3):
            for x in range(4):
                assert b[i, y, x] == pytest.approx(float(f[i, 2 * y:2 * y + 2, 2 * x:2 * x + 2].astype(np.float64).sum()),
                                                   rel=1e-15, abs=1e-15)
    e = f[:, :6, :8]
    assert np.allclose(prep.bin2x2(e).sum(axis=(1, 2)), e.astype(np.float64).sum(axis=(1, 2)), rtol=1e-13)


def test_planted_mean_instead_of_median_is_caught(monkeypatch):
    monkeypatch.setattr(prep, "median_subtract",
                        lambda f: (np.asarray(f, np.float64) - np.asarray(f, np.float64).mean(axis=0)[None],
                                   np.asarray(f, np.float64).mean(axis=0)))
    with pytest.raises(AssertionError):
        test_median_hand_values()


def test_planted_bin_mean_is_caught(monkeypatch):
    real = prep.bin2x2
    monkeypatch.setattr(prep, "bin2x2", lambda f: real(f) / 4.0)
    with pytest.raises(AssertionError):
        test_bin2x2_bruteforce_and_conservation()
