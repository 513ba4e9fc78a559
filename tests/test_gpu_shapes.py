"""Velocity-block shapes and the shape tuner (through the C ABI).

Every compiled shape must give the candidate lists of the default shape bit
for bit (the per-pixel sums are the same float32 additions in frame order,
only the grouping of velocities into workgroups differs); the tuner must
return a plan with one of them, remember its choice per geometry, and a
batch may mix plans of different shapes.
"""

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


CASES = [(50, 10, 70, 130, 7, 5, 3.0), (51, 16, 64, 64, 6, 4, 2.0), (52, 8, 33, 97, 5, 9, 6.0),
         (53, 12, 97, 61, 6, 4, 4.0), (55, 24, 128, 128, 13, 11, 5.0), (56, 9, 100, 150, 4, 25, 1.0)]


def _fields():
    out = [synth.tiny_field()]
    for seed, n, h, w, nvx, nvy, vmax in CASES:
        out.append(synth.small_case(seed, n, h, w, nvx, nvy, vmax=vmax, sky=50.0, sigma=5.0))
    return out


def test_shapes_listed(sst):
    shapes = sst.sst_shapes()
    assert shapes[:3] == [(6, 2), (6, 2), (12, 2)]
    for vbx, vby in shapes:
        # one pair of y velocities per block, three x velocities per wave
        assert vby == 2 and vbx % 3 == 0


def test_every_shape_matches_default(sst):
    nsh = len(sst.sst_shapes())
    for f in _fields():
        thr, kmax = (f.threshold, f.k_max) if f.n == 32 else (2.5, 8)
        fr = torch.from_numpy(f.frames).to("cuda:0")
        c0, n0 = sst.sst_detect(fr, f.t, f.t_ref, f.vx, f.vy, thr, f.min_coverage, kmax)
        for sh in range(nsh):
            plan = sst.sst_plan_detect(f.n, f.h, f.w, f.t, f.t_ref, f.vx, f.vy, thr, f.min_coverage, kmax, shape=sh)
            c, n = plan.run(fr)
            torch.cuda.synchronize()
            assert torch.equal(c, c0) and torch.equal(n, n0), (f.name, sh)
            _say(f"case {f.name}: shape {sh} ({'staged' if plan.staged else 'direct'}) matches the default, "
                 f"{int(n0.sum())} candidates")
            plan.close()


def test_tuner_picks_a_shape_and_remembers_it(sst):
    f = synth.tiny_field()
    fr = torch.from_numpy(f.frames).to("cuda:0")
    plan = sst.tune_plan(fr, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max)
    sh = sst.tuned_shape(f.n, f.h, f.w, f.t, f.t_ref, f.vx, f.vy, f.k_max)
    times = sst.tuning_times(f.n, f.h, f.w, f.t, f.t_ref, f.vx, f.vy, f.k_max)
    _say(f"case tuner on {f.name}: shape {sh}, ms per run by shape {times}")
    assert sh == plan.shape and len(times) == len(sst.sst_shapes())
    assert times[sh] == min(times)
    c, n = plan.run(fr)
    c0, n0 = sst.sst_detect(fr, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max)
    torch.cuda.synchronize()
    assert torch.equal(c, c0) and torch.equal(n, n0)
    again = sst.tune_plan(fr, f.t, f.t_ref, f.vx, f.vy, f.threshold, f.min_coverage, f.k_max)
    assert again.shape == sh
    plan.close()
    again.close()


def test_batch_of_mixed_shapes(sst):
    fields = _fields()
    plans, frames, ref = [], [], []
    for k, f in enumerate(fields):
        thr, kmax = (f.threshold, f.k_max) if f.n == 32 else (2.5, 8)
        fr = torch.from_numpy(f.frames).to("cuda:0")
        plans.append(sst.sst_plan_detect(f.n, f.h, f.w, f.t, f.t_ref, f.vx, f.vy, thr, f.min_coverage, kmax,
                                         shape=k % len(sst.sst_shapes())))
        frames.append(fr)
        ref.append(sst.sst_detect(fr, f.t, f.t_ref, f.vx, f.vy, thr, f.min_coverage, kmax))
    batch = sst.SstBatch(plans)
    cands, counts = batch.run(frames)
    torch.cuda.synchronize()
    for k, (c0, n0) in enumerate(ref):
        assert torch.equal(cands[k], c0) and torch.equal(counts[k], n0), k
    _say(f"case batch of {len(plans)} fields in every shape matches sst_detect")
    batch.close()
    for p in plans:
        p.close()
