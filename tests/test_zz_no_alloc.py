"""sst_detect_noalloc (the library's static scratch as workspace) against
sst_detect (a caller's workspace), through the C ABI: two calls in a row, the
second on a smaller problem, each giving sst_detect's lists and counts bit
for bit (the same kernels on the same inputs); a problem larger than the
scratch is rejected before any device work."""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def _run_both(sst, f, thr, kmax):
    fr = torch.from_numpy(f.frames).to("cuda:0")
    nk = len(f.vx) * len(f.vy)
    cand = torch.full((nk, kmax, 8), -7, dtype=torch.int32, device="cuda:0")
    count = torch.full((nk,), -7, dtype=torch.int32, device="cuda:0")
    sst.sst_detect_noalloc(fr, f.t, f.t_ref, f.vx, f.vy, thr, 0, kmax, cand, count)
    c2, n2 = sst.sst_detect(fr, f.t, f.t_ref, f.vx, f.vy, thr, 0, kmax)
    torch.cuda.synchronize()
    assert torch.equal(cand, c2) and torch.equal(count, n2)
    return int(count.sum().item())


def test_noalloc_matches_detect_twice_then_smaller(sst):
    big = synth.tiny_field()
    _say(f"case no-alloc {big.name}")
    n1 = _run_both(sst, big, big.threshold, big.k_max)
    small = synth.small_case(7, 9, 70, 90, 5, 4, vmax=3.0, sky=20.0, sigma=3.0)
    _say(f"case no-alloc {small.name} (second, smaller)")
    n2 = _run_both(sst, small, 3.0, 8)
    _say(f"  candidates: {n1} then {n2}; scratch {sst.sst_noalloc_scratch_bytes()} bytes")
    assert n1 > 0 and n2 > 0


def test_noalloc_two_passes_forced(sst):
    """The same two calls with the two-pass search forced (its counters and
    marks then live in the scratch too), against sst_detect in one pass."""
    from paper_2303_07293_amd import binding as B

    prev = B.sst_set_two_pass(B.SST_TWO_PASS_ALWAYS)
    try:
        for f, thr, kmax in ((synth.tiny_field(), None, None),
                             (synth.small_case(7, 9, 70, 90, 5, 4, vmax=3.0, sky=20.0, sigma=3.0), 3.0, 8)):
            thr = f.threshold if thr is None else thr
            kmax = f.k_max if kmax is None else kmax
            _say(f"case no-alloc two passes {f.name}")
            fr = torch.from_numpy(f.frames).to("cuda:0")
            nk = len(f.vx) * len(f.vy)
            cand = torch.full((nk, kmax, 8), -7, dtype=torch.int32, device="cuda:0")
            count = torch.full((nk,), -7, dtype=torch.int32, device="cuda:0")
            sst.sst_detect_noalloc(fr, f.t, f.t_ref, f.vx, f.vy, thr, 0, kmax, cand, count)
            torch.cuda.synchronize()
            B.sst_set_two_pass(B.SST_TWO_PASS_NEVER)
            c2, n2 = sst.sst_detect(fr, f.t, f.t_ref, f.vx, f.vy, thr, 0, kmax)
            torch.cuda.synchronize()
            B.sst_set_two_pass(B.SST_TWO_PASS_ALWAYS)
            assert torch.equal(cand, c2) and torch.equal(count, n2)
            assert int(count.sum().item()) > 0
    finally:
        B.sst_set_two_pass(prev)


def test_noalloc_rejects_problems_larger_than_the_scratch(sst):
    f = synth.full_field(n_movers=0, h=64, w=64)  # the grid and frames only set the size below
    n, h, w = 64, 1024, 1024
    need = sst.sst_workspace_bytes(sst.SST_OP_DETECT, n, h, w, f.t, f.t_ref, f.vx, f.vy, 64)
    assert need > sst.sst_noalloc_scratch_bytes()
    fr = torch.empty((n, h, w), dtype=torch.float32, device="cuda:0")
    nk = len(f.vx) * len(f.vy)
    cand = torch.empty((nk, 64, 8), dtype=torch.int32, device="cuda:0")
    count = torch.empty((nk,), dtype=torch.int32, device="cuda:0")
    with pytest.raises(sst.SstError) as e:
        sst.sst_detect_noalloc(fr, f.t, f.t_ref, f.vx, f.vy, 5.0, 0, 64, cand, count)
    assert e.value.code == -4 and "static scratch" in str(e.value)
