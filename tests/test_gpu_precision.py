"""16-bit frame storage on the GPU (through the C ABI).

* the quantiser (scales and 16-bit words) is bit-exact against the oracle's;
* statistics, stacks and candidate lists computed from 16-bit frames obey the
  same parity rules as float32 frames, against the float64 oracle run on the
  oracle's own dequantised frames F' = scale_i * q;
* on the full field, the error of 16-bit storage against the float64 oracle
  on the original float32 frames is measured and bounded by the format's
  unit roundoff, and detections are compared with the float32 GPU path
  over the whole grid and with the float64 oracle on the original frames on
  sampled velocities (every decision outside a guard band of 6 times the
  measured rms S/N error of the format must match).
"""

import sys

import numpy as np
import pytest

import oracle
from oracle import sst_oracle as so
import synth
from parity import SAFETY, U, compare_velocity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KINDS = {"bf16": ("bfloat16", 2.0 ** -8), "f16": ("float16", 2.0 ** -11)}


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


def _tdtype(kind):
    return getattr(torch, KINDS[kind][0])


def _upload_q(q, kind):
    return torch.from_numpy(np.ascontiguousarray(q).view(np.int16)).to("cuda:0").view(_tdtype(kind))


@pytest.mark.parametrize("kind", ["bf16", "f16"])
@pytest.mark.parametrize("center", [False, True])
def test_quantize_bit_exact(sst, kind, center):
    rng = np.random.default_rng(5)
    f = rng.normal(100, 10, size=(5, 37, 203)).astype(np.float32)
    f[1] = rng.normal(0, 1e-3, size=f[1].shape)
    f[2] = 0.0
    # frame 3: max 2^14 gives scale 1, so these values are exact rounding ties
    f[3] = 1.0
    f[3, 0, 0] = 2.0 ** 14
    f[3, 1, :4] = [1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -11, -(1 + 3 * 2 ** -11)]
    f[4] = rng.uniform(-5, 5, size=f[4].shape)
    _say(f"case quantize {kind} center={center}")
    q, s, o = sst.sst_quantize(torch.from_numpy(f).to("cuda:0"), _tdtype(kind), center=center)
    torch.cuda.synchronize()
    qw, sw, ow = oracle.quantize_frames(f, kind, center=center)
    assert np.array_equal(o.cpu().numpy(), ow)
    assert np.array_equal(s.cpu().numpy(), sw)
    got = q.cpu().view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, qw), int((got != qw).sum())


@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_stats_and_stack_16bit(sst, kind):
    f = synth.small_case(41, 7, 70, 130, 7, 5, vmax=3.0, sky=100.0, sigma=10.0)
    _say(f"case {f.name} {kind}")
    q, s, _ = oracle.quantize_frames(f.frames, kind)
    fd = oracle.dequantize_frames(q, s, kind)
    qt = _upload_q(q, kind)
    st = torch.from_numpy(s).to("cuda:0")
    stats = sst.sst_frame_stats(qt, scale=st).cpu().numpy()
    b, s2 = oracle.frame_stats(fd)
    assert np.allclose(stats[:, 0], b, rtol=1e-13) and np.allclose(stats[:, 1], s2, rtol=1e-11)
    out, cov = sst.sst_stack(qt, f.t, f.t_ref, f.vx, f.vy, with_coverage=True, scale=st)
    torch.cuda.synchronize()
    dx = oracle.shift_table(f.t, f.t_ref, f.vx)
    dy = oracle.shift_table(f.t, f.t_ref, f.vy)
    for k in range(len(f.vx) * len(f.vy)):
        a, bb = k % len(f.vx), k // len(f.vx)
        S, c, _, A = so.stack_velocity(fd, dx[:, a], dy[:, bb], absolute=True)
        assert np.array_equal(cov[bb, a].cpu().numpy(), c)
        err = np.abs(out[bb, a].cpu().numpy().astype(np.float64) - S)
        assert np.all(err <= 1e-5 * A + 1e-30), k


def _half_extra(f, fd, ks):
    """Extra flux bound of the search on IEEE-half samples, per velocity k.
    That search adds fma(q, scale, S) in float32 (each step one rounding of
    a partial sum bounded by sum |F'|, F' = scale q) and subtracts the
    covering frames' means once at the end, so besides the float32 bound of
    the oracle's own terms it may differ by (N + 2) u sum |F'| (the oracle's
    F' are float32 products: one more u |F'| per term, and the final
    subtraction)."""
    dx = oracle.shift_table(f.t, f.t_ref, f.vx)
    dy = oracle.shift_table(f.t, f.t_ref, f.vy)
    out = {}
    for k in ks:
        a, bb = k % len(f.vx), k // len(f.vx)
        A_raw = so.stack_velocity(fd, dx[:, a], dy[:, bb], absolute=True)[3]
        out[k] = SAFETY * (f.n + 2) * U * A_raw
    return out


@pytest.mark.parametrize("kind", ["bf16", "f16", "f16-direct"])
@pytest.mark.parametrize("center", [False, True])
def test_detect_16bit(sst, kind, center):
    direct = kind == "f16-direct"
    kind = "f16" if direct else kind
    f = synth.small_case(42, 12, 97, 61, 6, 4, vmax=4.0, sky=100.0, sigma=2.0)
    _say(f"case {f.name} {kind} center={center} search on 16-bit samples: {direct}")
    prev = sst.sst_set_half_search(direct)
    q, s, _ = oracle.quantize_frames(f.frames, kind, center=center)
    fd = oracle.dequantize_frames(q, s, kind)
    try:
        cand, count = sst.sst_detect(_upload_q(q, kind), f.t, f.t_ref, f.vx, f.vy, 2.5, 0, 6,
                                     scale=torch.from_numpy(s).to("cuda:0"))
        torch.cuda.synchronize()
    finally:
        sst.sst_set_half_search(prev)
    got = sst.candidates_to_numpy(cand)
    cnt = count.cpu().numpy()
    nvx = len(f.vx)
    ks = list(range(nvx * len(f.vy)))
    ref = oracle.detect(fd, f.t, f.t_ref, f.vx, f.vy, 2.5, 0, 6, velocities=ks, keep_maps=True)
    b, _ = oracle.frame_stats(fd)
    extra = _half_extra(f, fd, ks) if direct else {k: 0.0 for k in ks}
    marg = sum(compare_velocity(got[k], int(cnt[k]), ref[k], f.n, float(np.abs(b).max()), 2.5, ref["c_min"], 6, f.w,
                                extra_flux=extra[k])
               for k in ks)
    _say(f"  {int(cnt.sum())} candidates, {marg} marginal decisions")
    assert marg <= (4 if center else 16)


@pytest.fixture
def half_search(sst):
    prev = sst.sst_set_half_search(True)
    yield
    sst.sst_set_half_search(prev)


@pytest.mark.parametrize("shape,keep", [(0, 0), (1, 0), (2, 0), (0, 2)])
def test_half_search_random_cases(sst, shape, keep, half_search):
    """The search on IEEE-half samples (staged plans read the 16-bit copy,
    scale each sample in a mixed-precision fma, subtract the backgrounds
    through the prefix of the means) against the float64 oracle on the
    dequantised frames: random small problems spanning several tiles and
    ragged tails, centred and raw storage, both window widths, plus one
    problem whose shifts are too spread for a staged window (the float32
    copy)."""
    rng = np.random.default_rng(900 + shape + 7 * keep)
    marg = listed = 0
    for case in range(6):
        n, h, w = int(rng.integers(3, 30)), int(rng.integers(20, 140)), int(rng.integers(30, 200))
        nvx, nvy = int(rng.integers(1, 13)), int(rng.integers(1, 9))
        vmax = 60.0 if case == 5 else float(rng.choice([0.5, 2.0, 5.0]))
        f = synth.small_case(950 + 10 * shape + case, n, h, w, nvx, nvy, vmax=vmax, sky=float(rng.choice([0.0, 80.0])),
                             sigma=3.0, ties=bool(case % 2))
        center = bool(rng.integers(0, 2))
        thr = float(rng.choice([1.5, 3.0]))
        kmax = int(rng.choice([3, 16]))
        q, s, _ = oracle.quantize_frames(f.frames, "f16", center=center)
        fd = oracle.dequantize_frames(q, s, "f16")
        prev = sst.sst_set_slot_keep(keep)  # 2: most velocities recomputed after the merge
        try:
            plan = sst.sst_plan_detect(n, h, w, f.t, f.t_ref, f.vx, f.vy, thr, 0, kmax, shape=shape)
        finally:
            sst.sst_set_slot_keep(prev)
        _say(f"case {case}: {f.name} f16 center={center} thr {thr} kmax {kmax} shape {shape} "
             f"({'staged' if plan.staged else 'direct'})")
        cand, count = plan.run(_upload_q(q, "f16"), scale=torch.from_numpy(s).to("cuda:0"))
        torch.cuda.synchronize()
        got = sst.candidates_to_numpy(cand)
        cnt = count.cpu().numpy()
        ks = list(range(nvx * nvy))
        ref = oracle.detect(fd, f.t, f.t_ref, f.vx, f.vy, thr, 0, kmax, velocities=ks, keep_maps=True)
        b, _ = oracle.frame_stats(fd)
        extra = _half_extra(f, fd, ks)
        for k in ks:
            marg += compare_velocity(got[k], int(cnt[k]), ref[k], n, float(np.abs(b).max()), thr, ref["c_min"], kmax,
                                     w, extra_flux=extra[k])
            listed += min(int(ref[k]["count"]), kmax)
        plan.close()
    _say(f"  {marg} marginal decisions, {listed} listed entries")
    assert marg <= 0.05 * listed + 8


def test_16bit_frames_need_scale(sst):
    x = torch.zeros((2, 8, 8), dtype=torch.bfloat16, device="cuda:0")
    with pytest.raises(ValueError):
        sst.sst_frame_stats(x)


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["bf16", "f16", "f16-direct"])
@pytest.mark.parametrize("center", [False, True])
def test_precision_full_field(sst, kind, center):
    """Full field stored in 16 bits.  Error of the background-subtracted
    stack S' (the quantity the S/N is made of) against the float64 oracle on
    the original float32 frames, its S/N error, and agreement of the
    candidate lists with the float32 path.  Bounds: every stored sample of
    F - o carries one rounding of relative size <= u (the format's unit
    roundoff) and each frame's mean moves by at most u max|F - o|, so
    |dS'| <= 2 u sum_i max|F_i - o_i| plus float32 summation terms."""
    direct = kind == "f16-direct"  # the search on the 16-bit samples themselves
    kind = "f16" if direct else kind
    f = synth.full_field()
    _say(f"case {f.name} {kind} center={center} search on 16-bit samples: {direct}")
    fr = torch.from_numpy(f.frames).to("cuda:0")
    q, s, o = sst.sst_quantize(fr, _tdtype(kind), center=center)
    u = KINDS[kind][1]
    st16 = sst.sst_frame_stats(q, scale=s).cpu().numpy()
    b64, s2_64 = oracle.frame_stats(f.frames)
    ov = o.cpu().numpy().astype(np.float64)
    M = np.abs(f.frames.reshape(f.n, -1).astype(np.float64) - ov[:, None]).max(axis=1)
    ks = [0, 80, 3280, 6480, 6560, 41 * 81 + 7, 1234, 4321]
    dx = oracle.shift_table(f.t, f.t_ref, f.vx)
    dy = oracle.shift_table(f.t, f.t_ref, f.vy)
    worst_b, worst_rel, sq, npx, worst_sn, sq_sn = 0.0, 0.0, 0.0, 0, 0.0, 0.0
    for k in ks:
        a, b = k % 81, k // 81
        out = sst.sst_stack(q, f.t, f.t_ref, f.vx[a:a + 1], f.vy[b:b + 1], bg=st16[:, 0], scale=s)
        torch.cuda.synchronize()
        S, c, V, A = so.stack_velocity(f.frames, dx[:, a], dy[:, b], offsets=b64, weights=s2_64, absolute=True)
        g = out[0, 0].cpu().numpy().astype(np.float64)
        err = np.abs(g - S)
        # in-frame samples of each pixel: the bound sums M over at most c frames
        bound = 2 * u * c * M.max() + 4 * f.n * 2.0 ** -24 * c * (np.abs(f.frames).max() + M.max()) + 1e-30
        worst_b = max(worst_b, float((err / bound).max()))
        m = c >= f.min_coverage
        rel = err[m] / A[m]
        worst_rel = max(worst_rel, float(rel.max()))
        sq += float((rel ** 2).sum())
        npx += int(m.sum())
        # the flux part of the S/N error (the variances move by O(u) relative)
        esn = err[m] / np.sqrt(V[m])
        worst_sn = max(worst_sn, float(esn.max()))
        sq_sn += float((esn ** 2).sum())
    rms = (sq / max(npx, 1)) ** 0.5
    rms_sn = (sq_sn / max(npx, 1)) ** 0.5
    _say(f"  S' error: max/bound {worst_b:.3g}; |dS'|/A' over c >= c_min: max {worst_rel:.3g} rms {rms:.3g}; "
         f"flux part of |dSN| max {worst_sn:.3g} rms {rms_sn:.3g} (u = {u:.3g})")
    assert worst_b <= 1.0
    # candidate lists of the 16-bit search against the float64 oracle on the
    # original float32 frames, on the sampled velocities: every decision
    # outside a guard band of 6 times the measured rms S/N error of the
    # storage format (on top of the float32 bounds) must match
    prev = sst.sst_set_half_search(direct)
    try:
        c16s, n16s = sst.sst_detect(q, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max, scale=s)
        c16, n16 = sst.sst_detect(q, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max, scale=s)
        torch.cuda.synchronize()
    finally:
        sst.sst_set_half_search(prev)
    g16s, n16s = sst.candidates_to_numpy(c16s), n16s.cpu().numpy()
    ref = oracle.detect(f.frames, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max, velocities=ks,
                        keep_maps=True)
    marg = 0
    for k in ks:
        guard = 6.0 * rms_sn * np.sqrt(np.where(ref[k]["V"] > 0, ref[k]["V"], 0.0))
        marg += compare_velocity(g16s[k], int(n16s[k]), ref[k], f.n, float(np.abs(b64).max()), f.threshold,
                                 ref["c_min"], f.k_max, f.w, extra_flux=guard)
    _say(f"  {kind} lists on {len(ks)} velocities against the float64 oracle: {int(n16s[ks].sum())} candidates, "
         f"{marg} decisions inside the guard band")
    assert marg <= (4 if center else 16)
    # detections: 16-bit against float32 storage, whole grid
    c32, n32 = sst.sst_detect(fr, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max)
    g16, g32 = sst.candidates_to_numpy(c16), sst.candidates_to_numpy(c32)
    n16, n32 = n16.cpu().numpy(), n32.cpu().numpy()

    def snmap(g, n):
        out = {}
        for k in range(len(n)):
            m = min(int(n[k]), f.k_max)
            for x, y, sn in zip(g[k]["x"][:m], g[k]["y"][:m], g[k]["snr"][:m]):
                out[(k, int(y), int(x))] = float(sn)
        return out

    m16, m32 = snmap(g16, n16), snmap(g32, n32)
    common = m16.keys() & m32.keys()
    dsn = max((abs(m16[key] - m32[key]) for key in common), default=0.0)
    diff = sorted(m16.keys() ^ m32.keys())
    only = sorted(m16.get(key, m32.get(key)) for key in diff)
    _say(f"  detections: float32 {len(m32)}, {kind} {len(m16)}, common {len(common)}, max |dSN| on common "
         f"{dsn:.3g}; S/N of the differing ones: {[round(v, 3) for v in only[:12]]}")
    # A detection can only flip where its S/N or a neighbour's moves across the
    # threshold or a tie.  S/N error bound: the S' bound over the smallest V a
    # candidate can have (c_min frames of the smallest variance), plus the
    # O(u) relative change of the variances.
    v_min = f.min_coverage * float(s2_64.min())
    sn_bound = (2 * u * f.n * M.max() + 4 * f.n * 2.0 ** -24 * f.n * np.abs(f.frames).max()) / np.sqrt(v_min)
    sn_bound += 2 * u * max(max(m32.values()), max(m16.values()))
    _say(f"  S/N error bound {sn_bound:.3g}; differing detections {len(only)}")
    assert dsn <= sn_bound
    # each differing detection sits within the bound of the threshold or of
    # one of its neighbours (float64 S/N of the original frames at 3x3 pixels).
    # Both lists are within sn_bound (16-bit) and a far smaller float32 bound
    # of the float64 S/N of every pixel; a detection can differ only if one
    # of its decisions does: S/N against the threshold (one value, margin <=
    # sn_bound) or against a neighbour (two values, each moved by up to
    # sn_bound, margin <= 2 sn_bound).  So 2 sn_bound is the derived limit.
    fr64 = f.frames.astype(np.float64)

    def sn_at(k, y, x):
        a, b = k % 81, k // 81
        if not (0 <= x < f.w and 0 <= y < f.h):
            return -np.inf
        xs, ys = x + dx[:, a], y + dy[:, b]
        ok = (xs >= 0) & (xs < f.w) & (ys >= 0) & (ys < f.h)
        if ok.sum() < f.min_coverage:
            return -np.inf
        idx = np.nonzero(ok)[0]
        sp = float(np.sum(fr64[idx, ys[idx], xs[idx]] - b64[idx]))
        return sp / float(np.sqrt(np.sum(s2_64[idx])))

    near = 0
    for k, y, x in diff:
        c0 = sn_at(k, y, x)
        nb = [sn_at(k, y + j, x + i) for j in (-1, 0, 1) for i in (-1, 0, 1) if i or j]
        gap = min([abs(c0 - f.threshold)] + [abs(c0 - v) for v in nb])
        assert gap <= 2 * sn_bound, ((k, y, x), c0, gap)
        near += gap <= 2 * dsn
    _say(f"  every differing detection is within the bound of the threshold or a neighbour "
         f"({near} of {len(diff)} within twice the largest S/N change seen)")
