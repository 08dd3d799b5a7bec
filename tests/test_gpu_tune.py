"""Launch shapes and the tuner. A shape changes only the layout of the work: the
list-kernel residency, the lanes per target and the side stream for the pair kernel
leave every result bit unchanged; the grid chunk width changes the order of the
spread's and the gather's sums (sub-lanes share a stencil when fewer than 64 right-hand
sides form a chunk), the gather's work-group size the grouping of the partial sums of
a_k and the matrix-core pair kernel (with its candidate split) the order of the
direct-space sums, so results then agree to rounding. Every shape must match the
oracle; a measured shape is stored in the cache file and taken from there by the next
plan with the same key."""
import json

import numpy as np
import pytest
import torch

import synth
from oracle import method as om

pytestmark = pytest.mark.gpu

A = synth.ANGSTROM_BOHR


@pytest.fixture(scope="module")
def water600():
    return synth.water_box(200, seed=11)


def _plan(s, tune, shape=None, cache=None, block=64, prec=1, forces=False, graph=False):
    import paper_2307_02278_amd as P
    ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
    prm = P.Params(real_cutoff=7.0 * A, grid=(24, 24, 24), n_probes=block, n_steps=12,
                   block=block, precision=prec, seed=12345, tune=tune, shape=shape,
                   tune_cache=cache, want_forces=forces, graph=graph)
    return P.Plan([ds], prm)


SHAPES = [dict(pair_wg_per_cu=0, pair_subsets=0, grid_chunk=0, overlap=1),
          dict(pair_wg_per_cu=0, pair_subsets=0, grid_chunk=0, overlap=0),
          dict(pair_wg_per_cu=1, pair_subsets=4, grid_chunk=64, overlap=1),
          dict(pair_wg_per_cu=2, pair_subsets=1, grid_chunk=0, overlap=0),
          dict(pair_wg_per_cu=3, pair_subsets=2, grid_chunk=64, overlap=2),
          dict(pair_wg_per_cu=0, pair_subsets=2, grid_chunk=32, overlap=2),
          dict(pair_wg_per_cu=1, pair_subsets=4, grid_chunk=16, overlap=1),
          dict(pair_wg_per_cu=0, pair_subsets=0, grid_chunk=0, overlap=1, gather_waves=8),
          dict(pair_wg_per_cu=2, pair_subsets=2, grid_chunk=64, overlap=2, gather_waves=8),
          dict(pair_wg_per_cu=0, pair_subsets=0, grid_chunk=0, overlap=1, spread_mode=1),
          dict(pair_wg_per_cu=3, pair_subsets=1, grid_chunk=0, overlap=0, spread_mode=1),
          dict(pair_wg_per_cu=0, pair_subsets=1, grid_chunk=0, overlap=1, pair_mode=1),
          dict(pair_wg_per_cu=2, pair_subsets=1, grid_chunk=0, overlap=2, pair_mode=1),
          dict(pair_wg_per_cu=0, pair_subsets=2, grid_chunk=0, overlap=1, pair_mode=1),
          dict(pair_wg_per_cu=0, pair_subsets=1, grid_chunk=0, overlap=2, pair_mode=2),
          dict(pair_wg_per_cu=2, pair_subsets=2, grid_chunk=0, overlap=1, pair_mode=2)]


def test_shapes_give_the_same_bits_and_match_the_oracle(water600):
    import paper_2307_02278_amd as P
    s = water600
    v = torch.randn(64, s.n, 3, dtype=torch.float64, generator=torch.Generator().manual_seed(1))
    res = []
    for sh in SHAPES:
        plan = _plan(s, P.TUNE_GIVEN, sh, forces=True)
        inf = plan.info(0)
        assert inf.shape_source == 3
        assert inf.shape.pair_subsets == sh["pair_subsets"]
        assert inf.shape.overlap == sh["overlap"]
        assert inf.shape.spread_mode == sh.get("spread_mode", 0)
        assert inf.shape.pair_mode == sh.get("pair_mode", 0)
        out = plan.matvec(v.cuda()).cpu()
        e, f = plan.execute(forces=True)
        plan.check()
        mode = inf.shape.pair_mode
        res.append((out, e.cpu(), f.cpu(), (inf.shape.grid_chunk or 64,
                                             inf.shape.gather_waves or 4, mode,
                                             inf.shape.pair_subsets if mode else 0)))
        plan.close()
    # the same chunk width, gather work-group and direct-space summation: the same bits
    for k in range(1, len(SHAPES)):
        same = [j for j in range(k) if res[j][3] == res[k][3]]
        for j in same[:1]:
            for a, b in zip(res[k][:3], res[j][:3]):
                assert torch.equal(a, b), (SHAPES[k], SHAPES[j])
    # every shape: the method's result
    plan = _plan(s, P.TUNE_OFF)
    inf = plan.info(0)
    op = om.Operator(s, om.MethodParams(tau=inf.tau, r_pair=inf.r_pair, grid=(24, 24, 24),
                                        order=inf.spline_order))
    want = op(v.permute(1, 2, 0)).permute(2, 0, 1)
    den = want.abs().amax(dim=(1, 2))
    for sh, (out, e, f, _) in zip(SHAPES, res):
        err = float(((out - want).abs().amax(dim=(1, 2)) / den).max())
        ferr = float((f - res[0][2]).abs().max() / res[0][2].abs().max())
        print(f"shape {sh}: matvec vs oracle {err:.2e}; forces vs first shape {ferr:.2e}")
        assert err < 1e-6
        assert ferr < 1e-6
        assert float(e[0]) == pytest.approx(float(res[0][1][0]), rel=1e-6)


def test_measured_shape_is_cached_and_reused(water600, tmp_path):
    import paper_2307_02278_amd as P
    s = water600
    cache = str(tmp_path / "shapes.jsonl")
    ref = _plan(s, P.TUNE_OFF)
    e0 = ref.execute()
    ref.check()
    first = _plan(s, P.TUNE_MEASURE, cache=cache)
    inf = first.info(0)
    assert inf.shape_source == 1 and inf.tune_ms > 0.0
    e1 = first.execute()
    first.check()
    lines = [json.loads(x) for x in open(cache)]
    assert len(lines) == 1
    assert lines[0]["key"].split("|")[1:] == ["N=600", "K=24x24x24", "p=6", "B=64", "prec=1",
                                              "forces=0", "batch=0"]
    assert lines[0]["grid_chunk"] == inf.shape.grid_chunk
    second = _plan(s, P.TUNE_MEASURE, cache=cache)
    inf2 = second.info(0)
    assert inf2.shape_source == 2
    for k in ("pair_wg_per_cu", "pair_subsets", "grid_chunk", "overlap", "gather_waves",
              "spread_mode", "pair_mode"):
        assert getattr(inf2.shape, k) == getattr(inf.shape, k)
    e2 = second.execute()
    second.check()
    # the cached shape gives the measured shape's bits; against the built-in shape the
    # measured one may differ in summation order (chunk, gather group, matrix cores)
    assert torch.equal(e2, e1)
    assert float(e1[0]) == pytest.approx(float(e0[0]), rel=1e-6)
    assert len(open(cache).readlines()) == 1
    # another key (float64, block 16) is measured and appended
    third = _plan(s, P.TUNE_MEASURE, cache=cache, block=16, prec=0)
    assert third.info(0).shape_source == 1
    assert len(open(cache).readlines()) == 2


def test_tuned_batch_plan_keeps_one_stream_per_system():
    """Batch plans run systems on their own streams and tune without the side stream;
    the tuned batch gives the same bits as the built-in shape."""
    import paper_2307_02278_amd as P
    systems = [synth.water_box(100, seed=21), synth.water_box(60, seed=22)]
    ds = [P.DeviceSystem(x.pos, x.cell, x.alpha, x.omega, x.rvdw) for x in systems]
    out = []
    for tune in (P.TUNE_OFF, P.TUNE_MEASURE):
        prm = P.Params(real_cutoff=7.0 * A, grid=(0, 0, 0), n_probes=16, n_steps=10, block=16,
                       precision=P.PREC_MIXED, seed=3, tune=tune)
        plan = P.Plan(ds, prm)
        for k in range(2):
            assert plan.info(k).shape.overlap == 0
        out.append(plan.execute().cpu())
        plan.check()
    assert torch.equal(out[0], out[1])
