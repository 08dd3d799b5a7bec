"""mbd_scs_noalloc (the screening solve on the library's fixed per-GPU scratch array)
called through the C ABI against mbd_scs (per-call workspace): the same results bit for
bit, on two calls in a row, the second on a smaller system, then again on the first;
requests beyond the scratch size fail before any device work."""
import ctypes as C

import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

A = synth.ANGSTROM_BOHR


def _plan(s):
    import paper_2307_02278_amd as P
    ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
    prm = P.Params(real_cutoff=9.0 * A, grid=(0, 0, 0), n_probes=4, n_steps=4, block=4,
                   precision=P.PREC_MIXED)
    return P.Plan([ds], prm)


def _call(lib, fn, plan, n, n_freq):
    from paper_2307_02278_amd import _lib as L
    out = torch.full((3, n), float("nan"), dtype=torch.float64, device="cuda")
    af = torch.full((n_freq, n), float("nan"), dtype=torch.float64, device="cuda")
    prm = L.MbdScsParams(n_freq, 0.6, 1e-10, 1000)
    inf = L.MbdScsInfo()
    code = getattr(lib, fn)(plan.handle, 0, C.byref(prm), C.c_void_p(out[0].data_ptr()),
                            C.c_void_p(out[1].data_ptr()), C.c_void_p(out[2].data_ptr()),
                            C.c_void_p(af.data_ptr()), C.byref(inf))
    return code, out.cpu(), af.cpu(), (inf.iterations, inf.max_rel_residual)


def test_noalloc_screening_matches_allocating_entry_point():
    from paper_2307_02278_amd import _lib as L
    lib = L.lib()
    big = synth.water_box(400, seed=31)      # 1200 atoms
    small = synth.water_box(90, seed=32)     # 270 atoms, 8 frequencies
    cases = [(big, 15), (small, 8), (big, 15)]
    plans = {id(big): _plan(big), id(small): _plan(small)}
    for k, (s, nf) in enumerate(cases):
        plan = plans[id(s)]
        c0, ref, reff, inf0 = _call(lib, "mbd_scs", plan, s.n, nf)
        c1, got, gotf, inf1 = _call(lib, "mbd_scs_noalloc", plan, s.n, nf)
        assert c0 == L.MBD_OK and c1 == L.MBD_OK, (k, c0, c1, lib.mbd_last_error())
        print(f"call {k}: {s.n} atoms, {nf} frequencies, {inf1[0]} iterations, "
              f"residual {inf1[1]:.2e}")
        assert torch.isfinite(got).all() and torch.isfinite(gotf).all()
        assert torch.equal(got, ref), k
        assert torch.equal(gotf, reff), k
        assert inf0 == inf1, k
    for p in plans.values():
        p.close()


def test_noalloc_rejects_a_workspace_beyond_its_scratch():
    from paper_2307_02278_amd import _lib as L
    lib = L.lib()
    s = synth.water_box(4000, seed=33)     # 12000 atoms x 16 frequencies > 64 MiB
    plan = _plan(s)
    code, out, _, _ = _call(lib, "mbd_scs_noalloc", plan, s.n, 15)
    assert code == L.MBD_E_ARG
    assert b"scratch" in lib.mbd_last_error()
    assert torch.isnan(out).all()            # nothing was written
    plan.close()
