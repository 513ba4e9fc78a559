"""Pins of the CPU oracle to facts fixed outside the oracle itself.

Each pin checks the oracle against something it does not compute by itself:
closed-form integers, a hand-worked example, exact rational arithmetic, an
independent pure-Python brute force (with decimal rounding), the plain frame
sum, the sqrt(N) noise law, and the closed form of a stacked Gaussian mover.
The planted-mistake tests at the end break the oracle on purpose (on the CPU)
and check that some pin catches each mistake.
"""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import sst_oracle as so
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------- O1 rounding --
RHA_CASES = [
    (0.5, 1), (-0.5, -1), (1.5, 2), (-1.5, -2), (2.5, 3), (-2.5, -3),
    (0.49999999999999994, 0), (-0.49999999999999994, 0), (0.0, 0), (-0.0, 0),
    (2.4999999999999996, 2), (-2.5000000000000004, -3), (1e-300, 0), (-1e-300, 0),
    (123456.5, 123457), (-123456.5, -123457), (4503599627370495.5, 4503599627370496),
    (-0.5000000000000001, -1), (0.7, 1), (-0.7, -1), (3.0, 3), (-3.0, -3),
]


def pin_rha():
    xs = np.array([c[0] for c in RHA_CASES])
    want = np.array([c[1] for c in RHA_CASES], dtype=np.int64)
    got = so.rha(xs)
    assert np.array_equal(got, want), list(zip(xs, got, want))


def test_rha_closed_form():
    pin_rha()


def _exact_round(fr: Fraction) -> int:
    """Round half away from zero of an exact rational."""
    a = abs(fr)
    q = math.floor(a)
    if a - q >= Fraction(1, 2):
        q += 1
    return q if fr >= 0 else -q


def test_shift_table_matches_exact_rationals_on_config_timestamps():
    """For the tiny config (t_i = i/31) and the full-field config (slots of
    4/70 h), every v*(t_i - t_ref) is at least 1/70 away from a half-integer
    (2vi - 31(2k+1) and 4vm - 35(2k+1) are odd), so the float64 product rounds
    like the exact rational product; the oracle must agree with exact
    rational rounding everywhere."""
    # tiny config: t_i = i/31, v in -10..10
    t1 = np.arange(32, dtype=np.float64) / 31.0
    v1 = np.arange(-10, 11, dtype=np.float64)
    d1 = so.shift_table(t1, t1[0], v1)
    for i in range(32):
        for a, v in enumerate(v1):
            exact = Fraction(int(v)) * Fraction(i, 31)
            assert abs(exact - math.floor(exact) - Fraction(1, 2)) >= Fraction(1, 62)
            assert d1[i, a] == _exact_round(exact)
    # full-field config: slots m*(4/70) with 7 dropped, v in -40..40
    rng = np.random.default_rng(synth.SEED_BASE + 2)
    t2 = synth.fields.full_field_times(rng)
    slots = np.rint(t2 / (4.0 / 70.0)).astype(int)
    v2 = np.arange(-40, 41, dtype=np.float64)
    d2 = so.shift_table(t2, t2[0], v2)
    for i, m in enumerate(slots):
        for a, v in enumerate(v2):
            exact = Fraction(int(v)) * Fraction(2 * (int(m) - int(slots[0])), 35)
            assert d2[i, a] == _exact_round(exact)


def test_shift_table_monotone_in_time():
    rng = np.random.default_rng(5)
    t = np.cumsum(rng.uniform(0.001, 0.3, size=200))
    v = rng.uniform(-50, 50, size=33)
    d = so.shift_table(t, float(t[77]), v)
    for a in range(len(v)):
        col = d[:, a]
        if v[a] >= 0:
            assert np.all(np.diff(col) >= 0)
        else:
            assert np.all(np.diff(col) <= 0)


# --------------------------------------------------------- hand example --
def _hand():
    with open(os.path.join(GOLDEN, "hand_example.json")) as f:
        g = json.load(f)
    frames = np.array(g["frames"], dtype=np.float32)
    return g, frames


def pin_hand_example():
    g, frames = _hand()
    b, s2 = so.frame_stats(frames)
    assert np.array_equal(b, np.array(g["mean"]))
    assert np.array_equal(s2, np.array(g["var"]))
    for case in g["cases"]:
        dx = so.shift_table(g["t"], g["t_ref"], [case["vx"]])[:, 0]
        dy = so.shift_table(g["t"], g["t_ref"], [case["vy"]])[:, 0]
        assert list(dx) == case["dx"] and list(dy) == case["dy"]
        out, cov = so.stack(frames, g["t"], g["t_ref"], [case["vx"]], [case["vy"]])
        assert np.array_equal(out[0, 0], np.array(case["S"], dtype=np.float64))
        assert np.array_equal(cov[0, 0], np.array(case["c"]))
    sc = g["snr_case"]
    dx = so.shift_table(g["t"], g["t_ref"], [sc["vx"]])[:, 0]
    dy = so.shift_table(g["t"], g["t_ref"], [sc["vy"]])[:, 0]
    m = so.snr_velocity(frames, dx, dy, b, s2)
    assert m["S"][sc["y"], sc["x"]] == sc["S_prime"]
    assert m["V"][sc["y"], sc["x"]] == sc["V"]
    assert m["SN"][sc["y"], sc["x"]] == sc["S_prime"] / math.sqrt(sc["V"])


def test_hand_example():
    pin_hand_example()


def test_mean_stack_of_hand_example():
    g, frames = _hand()
    out, cov = so.stack(frames, g["t"], g["t_ref"], [1.0], [0.0], mode="mean")
    S = np.array(g["cases"][0]["S"], dtype=np.float64)
    c = np.array(g["cases"][0]["c"])
    assert np.array_equal(out[0, 0], S / c)


# --------------------------------------------------- O5/O6 hand SN images --
SN_IMG = np.array([[1, 5, 5, 0, 2],
                   [0, 0, 0, 0, 6],
                   [7, 0, 3, 3, 0],
                   [0, 0, 3, 3, 9]], dtype=np.float64)


def pin_candidate_rules():
    c = np.full(SN_IMG.shape, 10)
    # worked by hand: 9@(4,3), 7@(0,2), 6@(4,1), 5@(1,0) (beats its equal
    # right neighbour), 3@(2,2) (lowest raster of the 2x2 plateau); the 2 at
    # (4,0) equals the threshold and is rejected; the second 5 and the other
    # plateau pixels lose to an earlier equal neighbour.
    ras = so.candidates_from_maps(SN_IMG, c, 2.0, 1)
    assert list(ras) == [19, 10, 9, 1, 12]
    c2 = c.copy()
    c2[2, 0] = 4
    ras = so.candidates_from_maps(SN_IMG, c2, 2.0, 5)
    assert list(ras) == [19, 9, 1, 12]
    # a flat image: only the raster-first pixel is a maximum
    flat = np.full((3, 4), 7.0)
    assert list(so.candidates_from_maps(flat, np.ones((3, 4), int), 0.0, 1)) == [0]
    # corners and borders only compare with in-grid neighbours
    edge = np.zeros((3, 3))
    edge[0, 0] = edge[2, 2] = 4.0
    assert list(so.candidates_from_maps(edge, np.ones((3, 3), int), 1.0, 1)) == [0, 8]
    # a maximum exactly at the threshold is rejected (strict SN > threshold)
    assert list(so.candidates_from_maps(edge, np.ones((3, 3), int), 4.0, 1)) == []


def test_candidate_rules():
    pin_candidate_rules()


# Ten isolated static peaks on a zero sky (3 identical frames, 12 x 9, the
# zero-velocity bin only): S' = 3 (F - b), V = 3 s2, so SN = sqrt(3) (F - b) /
# sqrt(s2) with b = 54 / 108 and s2 = 366 / 108 - b^2 worked out by hand.
TRUNC_PEAKS = [((1, 1), 5), ((4, 1), 9), ((7, 1), 3), ((10, 1), 9), ((1, 4), 7),
               ((4, 4), 1), ((7, 4), 6), ((10, 4), 4), ((1, 7), 8), ((4, 7), 2)]


def pin_truncation_and_count():
    """O6: detect keeps the k_max best keys in key order, ranks them 0..k-1
    and counts every candidate before truncation."""
    h, w = 9, 12
    img = np.zeros((h, w), np.float32)
    for (x, y), v in TRUNC_PEAKS:
        img[y, x] = v
    frames = np.stack([img] * 3)
    t = np.array([0.0, 0.5, 1.0])
    b = Fraction(54, 108)
    s2 = Fraction(366, 108) - b * b
    # heights 4 and up clear SN 3 (SN(4) = 3.42, SN(3) = 2.44): 7 candidates;
    # key order 9 (raster 16), 9 (raster 22, the tie goes to the lower index),
    # 8 (85), 7 (49), 6 (55), 5 (13), 4 (58)
    want = [16, 22, 85, 49, 55, 13, 58]
    for k_max in (1, 4, 7, 10):
        out = so.detect(frames, t, 0.0, [0.0], [0.0], 3.0, 0, k_max)
        e = out[0]
        assert e["count"] == 7
        got = e["cand"]
        nk = min(k_max, 7)
        assert len(got) == nk
        assert list(got["y"] * w + got["x"]) == want[:nk]
        assert list(got["rank"]) == list(range(nk))
        assert np.all(got["coverage"] == 3) and np.all(got["ivx"] == 0) and np.all(got["ivy"] == 0)
        for r in got:
            v = int(img[r["y"], r["x"]])
            assert r["flux"] == pytest.approx(float(3 * (v - b)), rel=1e-14)
            assert r["snr"] == pytest.approx(math.sqrt(3.0) * float(v - b) / math.sqrt(float(s2)), rel=1e-12)


def test_truncation_and_count():
    pin_truncation_and_count()


# ------------------------------------------------------- O3 brute force --
@pytest.mark.parametrize("seed", range(8))
def test_brute_force_agrees_bitwise(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 7))
    h, w = int(rng.integers(1, 10)), int(rng.integers(1, 10))
    nvx, nvy = int(rng.integers(1, 4)), int(rng.integers(1, 4))
    f = synth.small_case(seed, n, h, w, nvx, nvy, vmax=4.0, sky=3.0, ties=(seed % 2 == 0))
    offs = rng.normal(3.0, 1.0, size=n)
    bf = so.brute_force_stack(f.frames, f.t, f.t_ref, f.vx, f.vy, offsets=offs)
    out, cov = so.stack(f.frames, f.t, f.t_ref, f.vx, f.vy, bg=offs)
    for b in range(nvy):
        for a in range(nvx):
            S, C = bf[b][a]
            assert np.array_equal(out[b, a], np.array(S)), (b, a)
            assert np.array_equal(cov[b, a], np.array(C)), (b, a)


def test_brute_force_covers_exact_ties():
    """Timestamps on a quarter-hour lattice and half-integer velocities make
    v*(t - t_ref) hit exact .5 values; the brute force's decimal rounding and
    the oracle must agree there."""
    f = synth.small_case(3, 6, 7, 8, 3, 3, vmax=3.0, ties=True)
    prods = np.abs((f.t - f.t_ref)[:, None] * f.vx[None, :])
    assert np.any(prods - np.floor(prods) == 0.5)
    bf = so.brute_force_stack(f.frames, f.t, f.t_ref, f.vx, f.vy)
    out, cov = so.stack(f.frames, f.t, f.t_ref, f.vx, f.vy)
    for b in range(3):
        for a in range(3):
            assert np.array_equal(out[b, a], np.array(bf[b][a][0]))
            assert np.array_equal(cov[b, a], np.array(bf[b][a][1]))


def test_raster_tie_rule_on_planted_pairs():
    """Isolated bright pixels are candidates; of two equal neighbours (equal
    values in every frame) only the one earlier in raster order is (Sec. 2.1
    peak rule as read here: earlier neighbours strictly smaller, later ones
    may tie).  The pairs sit across tile borders so that the GPU test of the
    same case covers the border evaluation."""
    f = synth.tile_border_case()
    ref = oracle.detect(f.frames, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max, velocities=[0])
    c, n = ref[0]["cand"], int(ref[0]["count"])
    found = set(zip(np.asarray(c["x"])[:n].tolist(), np.asarray(c["y"])[:n].tolist()))
    for p in synth.BORDER_PEAKS:
        assert p in found, p
    for first, second in synth.BORDER_TIES:
        assert first in found and second not in found, (first, second)


# ------------------------------------------------------ O3 zero velocity --
def pin_zero_velocity():
    rng = np.random.default_rng(11)
    frames = (rng.normal(100, 10, size=(9, 13, 17))).astype(np.float32)
    t = np.cumsum(rng.uniform(0.1, 0.5, size=9))
    out, cov = so.stack(frames, t, float(t[4]), [0.0], [0.0])
    seq = np.zeros((13, 17))
    for i in range(9):
        seq = seq + frames[i].astype(np.float64)
    assert np.array_equal(out[0, 0], seq)
    assert np.all(cov[0, 0] == 9)
    exact = so.fsum_frames(frames)
    ulp = np.spacing(np.abs(exact))
    assert np.all(np.abs(out[0, 0] - exact) <= 9 * ulp)


def test_zero_velocity_is_plain_frame_sum():
    pin_zero_velocity()


# ---------------------------------------------------------- O3/O4 noise --
def pin_noise_law():
    """Pure noise: the stack of N frames has variance N sigma^2 and the S/N
    has mean 0 and variance 1 (the sqrt(N) law behind stacking, Sec. 1)."""
    f = synth.pure_noise(0, 24, 128, 128, sigma=3.0, sky=50.0)
    b, s2 = so.frame_stats(f.frames)
    dx = so.shift_table(f.t, f.t_ref, [2.0])[:, 0]
    dy = so.shift_table(f.t, f.t_ref, [-1.0])[:, 0]
    m = so.snr_velocity(f.frames, dx, dy, b, s2)
    full = m["c"] == 24
    S = m["S"][full]
    assert abs(S.var() / (24 * 9.0) - 1) < 0.05
    sn = m["SN"][full]
    assert abs(sn.mean()) < 0.05
    assert abs(sn.var() - 1) < 0.05


def test_noise_law():
    pin_noise_law()


# ---------------------------------------------------------------- movers --
def pin_mover_closed_form():
    """Noise-free single mover with integer velocity and start pixel: the
    stack at (v_true, p0) equals sum_i A exp(-|r_i|^2 / 2s^2), r_i = v tau_i
    - d_i being each frame's sub-pixel residual of the integer shift; and the
    maximum of the whole stack cube is exactly at (v_true, p0)."""
    n, h, w = 16, 48, 48
    t = np.linspace(0.0, 2.0, n)
    mv = synth.Mover(20.0, 25.0, 3.0, -2.0, 5.0, 2.5)
    frames = np.zeros((n, h, w), np.float32)
    for i in range(n):
        img = np.zeros((h, w))
        synth.render_movers(img, float(t[i]), [mv])
        frames[i] = img.astype(np.float32)
    grid = np.arange(-4, 5, dtype=np.float64)
    out, cov = so.stack(frames, t, 0.0, grid, grid)
    b, a = 4 + (-2), 4 + 3
    s = mv.fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    want = 0.0
    for i in range(n):
        rx = 3.0 * t[i] - _exact_round(Fraction(3.0) * Fraction(float(t[i])))
        ry = -2.0 * t[i] - _exact_round(Fraction(-2.0) * Fraction(float(t[i])))
        want += float(np.float32(5.0 * math.exp(-(rx * rx + ry * ry) / (2 * s * s))))
    got = out[b, a, 25, 20]
    assert abs(got - want) <= 1e-6 * want, (got, want)
    flat = np.argmax(out)
    assert np.unravel_index(flat, out.shape) == (b, a, 25, 20)


def test_mover_closed_form_and_argmax():
    pin_mover_closed_form()


@pytest.mark.slow
def test_tiny_config_movers_recovered():
    """Tiny config with noise (A = 1.5 sigma, 32 frames over 1 h): at the true
    velocity bin and start pixel each mover's S/N is within 3.5 of its
    closed-form expectation sum_i A g_i / sqrt(N sigma^2) (about A sqrt(N) /
    sigma = 8.5 less the sub-pixel residual loss), and the best S/N within
    +-2 bins and +-3 px clears the 5 sigma threshold.  Over a 1 h baseline
    neighbouring 1 px/h bins differ by under a pixel, so with noise the
    maximum may sit one bin away; exact recovery is pinned noise-free above."""
    f = synth.tiny_field()
    dx = so.shift_table(f.t, f.t_ref, f.vx)
    dy = so.shift_table(f.t, f.t_ref, f.vy)
    b, s2 = so.frame_stats(f.frames)
    s = 2.5 / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    for mv in f.movers:
        ia0, ib0 = int(mv.vx) + 10, int(mv.vy) + 10
        sig = 0.0
        for ti in f.t:
            rx = mv.vx * ti - _exact_round(Fraction(mv.vx) * Fraction(float(ti)))
            ry = mv.vy * ti - _exact_round(Fraction(mv.vy) * Fraction(float(ti)))
            sig += mv.amp * math.exp(-(rx * rx + ry * ry) / (2 * s * s))
        expect = sig / math.sqrt(f.n * 1.0)
        m = so.snr_velocity(f.frames, dx[:, ia0], dy[:, ib0], b, s2)
        at_truth = m["SN"][int(mv.y0), int(mv.x0)]
        assert abs(at_truth - expect) < 3.5, (at_truth, expect, mv)
        best = -np.inf
        for ib in range(max(0, ib0 - 2), min(21, ib0 + 3)):
            for ia in range(max(0, ia0 - 2), min(21, ia0 + 3)):
                m = so.snr_velocity(f.frames, dx[:, ia], dy[:, ib], b, s2)
                y0, x0 = int(mv.y0), int(mv.x0)
                best = max(best, m["SN"][y0 - 3:y0 + 4, x0 - 3:x0 + 4].max())
        assert best > 5.0


def test_detect_finds_injected_mover_in_candidate_list():
    n, h, w = 20, 40, 40
    rng = np.random.default_rng(7)
    t = np.linspace(0.0, 1.0, n)
    mv = synth.Mover(15.0, 22.0, -4.0, 3.0, 4.0, 2.5)
    frames = np.empty((n, h, w), np.float32)
    for i in range(n):
        img = rng.normal(10.0, 1.0, size=(h, w))
        synth.render_movers(img, float(t[i]), [mv])
        frames[i] = img.astype(np.float32)
    grid = np.arange(-5, 6, dtype=np.float64)
    k = (3 + 5) * 11 + (-4 + 5)
    res = oracle.detect(frames, t, 0.0, grid, grid, 5.0, 0, 4, velocities=[k])
    top = res[k]["cand"][0]
    assert (top["x"], top["y"]) == (15, 22)
    assert top["coverage"] == n and top["rank"] == 0
    assert top["snr"] > 10


# ------------------------------------------------- planted mistakes (CPU) --
def _must_fail(pin):
    with pytest.raises(AssertionError):
        pin()


def test_planted_half_to_even_rounding_is_caught(monkeypatch):
    monkeypatch.setattr(so, "rha", lambda x: np.rint(np.asarray(x, np.float64)).astype(np.int64))
    _must_fail(pin_rha)


def test_planted_floor_plus_half_rounding_is_caught(monkeypatch):
    monkeypatch.setattr(so, "rha", lambda x: np.floor(np.asarray(x, np.float64) + 0.5).astype(np.int64))
    _must_fail(pin_rha)


def test_planted_shift_sign_flip_is_caught(monkeypatch):
    real = so.shift_table
    monkeypatch.setattr(so, "shift_table", lambda t, tr, v: -real(t, tr, v))
    _must_fail(pin_mover_closed_form)
    _must_fail(pin_hand_example)


def test_planted_sample_variance_is_caught(monkeypatch):
    def bad(frames):
        f = frames.reshape(frames.shape[0], -1).astype(np.float64)
        return f.mean(axis=1), f.var(axis=1, ddof=1)
    monkeypatch.setattr(so, "frame_stats", bad)
    _must_fail(pin_hand_example)


def test_planted_missing_background_is_caught(monkeypatch):
    real = so.stack_velocity

    def no_bg(frames, dx, dy, offsets=None, weights=None, absolute=False):
        return real(frames, dx, dy, None, weights, absolute)
    monkeypatch.setattr(so, "stack_velocity", no_bg)
    _must_fail(pin_noise_law)


def test_planted_tie_rule_reversed_is_caught(monkeypatch):
    def bad(sn):
        h, w = sn.shape
        P = np.full((h + 2, w + 2), -np.inf)
        P[1:-1, 1:-1] = sn
        ok = np.ones((h, w), dtype=bool)
        for ddy in (-1, 0, 1):
            for ddx in (-1, 0, 1):
                if ddx == 0 and ddy == 0:
                    continue
                q = P[1 + ddy:1 + ddy + h, 1 + ddx:1 + ddx + w]
                earlier = ddy < 0 or (ddy == 0 and ddx < 0)
                ok &= (sn >= q) if earlier else (sn > q)
        return ok
    monkeypatch.setattr(so, "local_max_mask", bad)
    _must_fail(pin_candidate_rules)


def test_planted_dropped_last_frame_is_caught(monkeypatch):
    real = so.stack_velocity

    def drop(frames, dx, dy, offsets=None, weights=None, absolute=False):
        return real(frames[:-1], dx[:-1], dy[:-1],
                    None if offsets is None else offsets[:-1],
                    None if weights is None else weights[:-1], absolute)
    monkeypatch.setattr(so, "stack_velocity", drop)
    _must_fail(pin_zero_velocity)


def test_planted_threshold_inclusive_is_caught(monkeypatch):
    real = so.candidates_from_maps

    def incl(sn, c, threshold, c_min):
        return real(sn, c, np.nextafter(threshold, -np.inf), c_min)
    monkeypatch.setattr(so, "candidates_from_maps", incl)
    _must_fail(pin_candidate_rules)


def test_planted_count_after_truncation_is_caught(monkeypatch):
    real = so.velocity_list

    def bad(ras, m, ia, ib, w, k_max):
        rec, _ = real(ras, m, ia, ib, w, k_max)
        return rec, len(rec)
    monkeypatch.setattr(so, "velocity_list", bad)
    _must_fail(pin_truncation_and_count)


def test_planted_one_based_rank_is_caught(monkeypatch):
    real = so.velocity_list

    def bad(ras, m, ia, ib, w, k_max):
        rec, cnt = real(ras, m, ia, ib, w, k_max)
        rec["rank"] += 1
        return rec, cnt
    monkeypatch.setattr(so, "velocity_list", bad)
    _must_fail(pin_truncation_and_count)


def test_planted_keep_last_k_is_caught(monkeypatch):
    real = so.velocity_list

    def bad(ras, m, ia, ib, w, k_max):
        return real(ras[::-1][:k_max][::-1] if len(ras) > k_max else ras, m, ia, ib, w, k_max)
    monkeypatch.setattr(so, "velocity_list", bad)
    _must_fail(pin_truncation_and_count)
