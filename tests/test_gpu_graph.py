"""Graph replay of mbd_execute: a plan created with graph=1 records its whole launch
sequence once (per variant) and replays it. Every replay must reproduce the eager
result bit for bit, with the program's own eager work and synchronizations between
replays, and after the positions change."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

A = synth.ANGSTROM_BOHR


def _systems():
    return [synth.workload("tiny").systems[0], synth.tiny_random(seed=9, n=40)]


def _plans(systems, prec, forces):
    import paper_2307_02278_amd as P
    ds = [P.DeviceSystem(x.pos, x.cell, x.alpha, x.omega, x.rvdw) for x in systems]
    kw = dict(ewald_tau=0.35 * synth.BOHR_ANGSTROM, real_cutoff=13.0 * A, grid=(16, 16, 16),
              n_probes=8, n_steps=10, block=8 if prec == P.PREC_FP64 else 16, precision=prec,
              seed=12345, want_forces=forces)
    eager = P.Plan(ds, P.Params(**kw))
    graph = P.Plan(ds, P.Params(graph=True, **kw))
    return eager, graph, ds


@pytest.mark.parametrize("prec,forces", [(0, True), (1, True), (1, False)])
def test_graph_replays_match_eager(prec, forces):
    import paper_2307_02278_amd as P
    systems = _systems()
    eager, graph, ds = _plans(systems, prec, forces)
    ref = eager.execute(forces=forces)
    eager.check()
    ref = [t.clone() for t in ref] if forces else [ref.clone()]
    other = torch.randn(4, systems[0].n, 3, dtype=torch.float64, device="cuda")
    for rep in range(4):
        out = graph.execute(forces=forces)
        graph.check()
        out = list(out) if forces else [out]
        for a, b in zip(out, ref):
            assert torch.equal(a, b), rep
        # eager work of the program between replays
        eager.matvec(other)
        _ = (other * 2.0).sum().item()
        torch.cuda.synchronize()


def test_graph_replay_follows_new_positions():
    import paper_2307_02278_amd as P
    systems = _systems()
    eager, graph, ds = _plans(systems, P.PREC_MIXED, True)
    graph.execute(forces=True)
    graph.check()
    rng = np.random.default_rng(3)
    for rep in range(2):
        for k, x in enumerate(systems):
            p = torch.as_tensor(x.pos + rng.normal(scale=0.05 * A, size=x.pos.shape)).cuda()
            eager.set_positions(p, k)
            graph.set_positions(p, k)
        e0, f0 = eager.execute(forces=True)
        e1, f1 = graph.execute(forces=True)
        eager.check()
        graph.check()
        assert torch.equal(e0, e1) and torch.equal(f0, f1), rep


def test_graph_plan_runs_eagerly_while_timing():
    import paper_2307_02278_amd as P
    eager, graph, _ = _plans(_systems(), P.PREC_MIXED, False)
    ref = eager.execute()
    graph.set_timing(True)
    e = graph.execute()
    graph.set_timing(False)
    graph.check()
    times = graph.stage_times()
    assert times["pair"][1] > 0 and times["lanczos"][1] > 0
    assert torch.equal(e, ref)
