"""GPU parity of the preprocessing steps (through the C ABI) against the
float64 oracle.  Tolerances follow the float32 arithmetic, u = 2^-24:
the median of an odd count is one of the samples (exact), of an even count
one float32 add and halving (<= u |a + b|); each output of median removal
adds one rounding of the subtraction; a co-add of g frames accumulates at
most (g - 1) u sum|F|; a 2x2 bin 2 u sum|F|."""

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
U = 2.0 ** -24


@pytest.fixture(scope="module")
def sst():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_07293_amd as m
    m.load()
    return m


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _frames(seed, n, h, w, ties=False):
    rng = np.random.default_rng(seed)
    f = rng.normal(100, 10, size=(n, h, w)).astype(np.float32)
    if ties:
        f = np.round(f / 5) * 5  # many equal values per pixel
        f[:, 0, :] = -0.0
        f[: n // 2, 1, :] = 0.0
    return f


# n <= 64 takes the register form of the kernel, larger n the LDS form
@pytest.mark.parametrize("n,h,w,ties", [(1, 3, 5, False), (7, 33, 70, False), (8, 33, 70, True),
                                        (40, 20, 70, True), (64, 17, 130, False), (65, 9, 40, True),
                                        (256, 5, 67, True), (13, 1, 1, False)])
def test_median_subtract(sst, n, h, w, ties):
    _say(f"case median n={n} {h}x{w} ties={ties}")
    f = _frames(n, n, h, w, ties)
    out, med = sst.sst_median_subtract(torch.from_numpy(f).to("cuda:0"), with_median=True)
    torch.cuda.synchronize()
    ro, rm = oracle.median_subtract(f)
    gm = med.cpu().numpy().astype(np.float64)
    if n % 2:
        assert np.array_equal(gm, rm)
    else:
        s = np.sort(f.astype(np.float64), axis=0)
        ab = np.abs(s[n // 2 - 1] + s[n // 2])
        assert np.all(np.abs(gm - rm) <= U * ab)
    err = np.abs(out.cpu().numpy().astype(np.float64) - ro)
    assert np.all(err <= U * np.abs(ro) + 2 * U * np.abs(rm)[None] + 1e-30)


def test_median_frame_limit(sst):
    f = torch.zeros((257, 2, 2), dtype=torch.float32, device="cuda:0")
    with pytest.raises(sst.SstError):
        sst.sst_median_subtract(f)


@pytest.mark.parametrize("n,group", [(26, 13), (27, 13), (5, 1), (9, 9), (64, 14)])
def test_coadd(sst, n, group):
    _say(f"case coadd n={n} group={group}")
    f = _frames(100 + n, n, 19, 45)
    t = np.cumsum(np.random.default_rng(n).uniform(0.01, 0.02, n))
    out, t_out = sst.sst_coadd(torch.from_numpy(f).to("cuda:0"), group, t)
    torch.cuda.synchronize()
    ro, rt = oracle.coadd(f, group, t)
    assert out.shape[0] == n // group
    ra, _ = oracle.coadd(np.abs(f), group)
    assert np.all(np.abs(out.cpu().numpy() - ro) <= (group - 1) * U * ra + 1e-30)
    assert np.allclose(t_out, rt, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n,h,w", [(3, 8, 8), (2, 9, 17), (1, 2, 2), (4, 1030, 514)])
def test_bin2x2(sst, n, h, w):
    _say(f"case bin {n}x{h}x{w}")
    f = _frames(200 + h, n, h, w)
    out = sst.sst_bin2x2(torch.from_numpy(f).to("cuda:0"))
    torch.cuda.synchronize()
    ro = oracle.bin2x2(f)
    assert tuple(out.shape) == ro.shape
    ra = oracle.bin2x2(np.abs(f))
    assert np.all(np.abs(out.cpu().numpy() - ro) <= 2 * U * ra + 1e-30)


def test_pipeline_static_sources_removed_before_search(sst):
    """Frames with bright static stars and one faint mover: after median
    removal on the GPU, the search finds the mover at its velocity bin and
    no star survives as a candidate."""
    rng = np.random.default_rng(77)
    n, h, w = 24, 96, 128
    t = np.arange(n) / (n - 1) * 2.0
    yy, xx = np.mgrid[0:h, 0:w]
    sky = np.zeros((h, w))
    for _ in range(12):
        sx, sy = rng.uniform(5, w - 5), rng.uniform(5, h - 5)
        sky += 500 * np.exp(-((xx - sx) ** 2 + (yy - sy) ** 2) / (2 * 1.2 ** 2))
    frames = np.empty((n, h, w), np.float32)
    x0, y0, vx, vy = 30.0, 40.0, 12.0, 6.0
    for i in range(n):
        img = sky + rng.normal(0, 1.0, size=(h, w))
        cx, cy = x0 + vx * t[i], y0 + vy * t[i]
        img += 4.0 * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * 1.06 ** 2))
        frames[i] = img
    fr = torch.from_numpy(frames).to("cuda:0")
    clean = sst.sst_median_subtract(fr)
    grid = np.arange(-15, 16, dtype=np.float64)
    cand, count = sst.sst_detect(clean, t, 0.0, grid, grid, 8.0, 0, 8)
    g = sst.candidates_to_numpy(cand)
    k = (int(vy) + 15) * 31 + int(vx) + 15
    assert int(count[k]) >= 1 and (g[k]["x"][0], g[k]["y"][0]) == (int(x0), int(y0))
    # the oracle agrees on the cleaned frames it computes itself
    ro, _ = oracle.median_subtract(frames)
    ref = oracle.detect(ro.astype(np.float32), t, 0.0, grid, grid, 8.0, 0, 8, velocities=[k])
    assert ref[k]["count"] >= 1 and (ref[k]["cand"]["x"][0], ref[k]["cand"]["y"][0]) == (int(x0), int(y0))
