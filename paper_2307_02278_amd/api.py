"""Python entry points over the C ABI. PyTorch supplies device memory and the
current HIP stream; every step of the computation runs in libmbd's kernels."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib as L


@dataclass
class Params:
    damp_beta: float = 0.83
    damp_d: float = 6.0
    ewald_tau: float = 0.0          # 1/bohr; 0 => from real_cutoff
    real_cutoff: float = 9.0 / 0.529177210903
    damp_tol: float = 0.0           # 0 => 1e-4
    grid: Sequence[int] = (0, 0, 0)
    spline_order: int = 6
    n_probes: int = 8
    n_steps: int = 30
    block: int = 0
    seed: int = 12345
    precision: int = L.PREC_FP64
    reorth: int = L.REORTH_NONE
    want_forces: bool = False
    graph: bool = False             # replay execute from a captured HIP graph
    replica_cutoff: float = 0.0     # bohr; > 0 => replica method (float64, energy only)
    krylov_block: int = 1           # > 1 => block Lanczos over blocks of this many probes
    tune: int = L.TUNE_OFF          # TUNE_OFF / TUNE_MEASURE / TUNE_GIVEN
    shape: Optional[dict] = None    # TUNE_GIVEN: mbd_shape fields (pair_wg_per_cu, pair_subsets,
    #                                 grid_chunk, overlap, gather_waves, spread_mode, pair_mode)
    tune_cache: Optional[str] = None  # TUNE_MEASURE: JSON-lines cache file
    store_grids: bool = False       # forces: keep the forward steps' potential grids

    def to_c(self) -> L.MbdParams:
        p = L.MbdParams()
        p.damp_beta = self.damp_beta
        p.damp_d = self.damp_d
        p.ewald_tau = self.ewald_tau
        p.real_cutoff = self.real_cutoff
        p.damp_tol = self.damp_tol
        g = list(self.grid) + [0] * (3 - len(self.grid))
        for a in range(3):
            p.grid[a] = int(g[a])
        p.spline_order = self.spline_order
        p.n_probes = self.n_probes
        p.n_steps = self.n_steps
        p.block = self.block
        p.seed = self.seed
        p.precision = self.precision
        p.reorth = self.reorth
        p.want_forces = 1 if self.want_forces else 0
        p.deterministic = 0
        p.graph = 1 if self.graph else 0
        p.replica_cutoff = self.replica_cutoff
        p.krylov_block = self.krylov_block
        p.tune = self.tune
        for k, v in (self.shape or {}).items():
            setattr(p.shape, k, int(v))
        self._cache_bytes = self.tune_cache.encode() if self.tune_cache else None
        p.tune_cache = self._cache_bytes
        p.store_grids = 1 if self.store_grids else 0
        return p


class DeviceSystem:
    """Device-resident copy of one periodic system (float64, atomic units)."""

    def __init__(self, pos, cell, alpha, omega, rvdw, device="cuda"):
        f = lambda x: torch.as_tensor(x, dtype=torch.float64).to(device).contiguous()
        self.pos = f(pos).reshape(-1, 3).contiguous()
        self.alpha = f(alpha)
        self.omega = f(omega)
        self.rvdw = f(rvdw)
        self.cell = [float(x) for x in torch.as_tensor(cell, dtype=torch.float64).reshape(9)]
        self.n = int(self.pos.shape[0])

    def to_c(self) -> L.MbdSystem:
        s = L.MbdSystem()
        s.n_atoms = self.n
        s.pos = self.pos.data_ptr()
        for i in range(9):
            s.cell[i] = self.cell[i]
        s.alpha = self.alpha.data_ptr()
        s.omega = self.omega.data_ptr()
        s.r_vdw = self.rvdw.data_ptr()
        return s


def _stream_ptr():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """Owns one mbd_plan. Systems must stay alive while the plan exists."""

    def __init__(self, systems: List[DeviceSystem], params: Params):
        self.lib = L.lib()
        self.systems = systems
        self.params = params
        arr = (L.MbdSystem * len(systems))(*[s.to_c() for s in systems])
        self._cparams = params.to_c()
        h = C.c_void_p()
        L.check(self.lib.mbd_plan_create(C.byref(h), arr, len(systems), C.byref(self._cparams),
                                         _stream_ptr()))
        self.handle = h

    def info(self, sys: int = 0) -> L.MbdInfo:
        inf = L.MbdInfo()
        L.check(self.lib.mbd_plan_info(self.handle, sys, C.byref(inf)))
        return inf

    def execute(self, forces: bool = False, energy_sd: bool = False):
        """E_MBD per system; with forces=True also F = -dE/dR, [sum N, 3]; with
        energy_sd=True also the standard deviation of each energy estimate (all float64,
        on the GPU). Returns e, or a tuple (e[, f][, sd]) in that order."""
        e = torch.zeros(len(self.systems), dtype=torch.float64, device="cuda")
        f = (torch.zeros(sum(s.n for s in self.systems), 3, dtype=torch.float64, device="cuda")
             if forces else None)
        sd = torch.zeros(len(self.systems), dtype=torch.float64, device="cuda") if energy_sd \
            else None
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        L.check(self.lib.mbd_execute(self.handle, ptr(e), ptr(f), ptr(sd)))
        if not forces and not energy_sd:
            return e
        return tuple(x for x in (e, f, sd) if x is not None)

    def check(self):
        L.check(self.lib.mbd_check(self.handle))

    def matvec(self, v: torch.Tensor, sys: int = 0, components: int = L.C_ALL) -> torch.Tensor:
        v = v.to(dtype=torch.float64, device="cuda").contiguous()
        squeeze = v.dim() == 2
        if squeeze:
            v = v[None]
        out = torch.empty_like(v)
        L.check(self.lib.mbd_matvec(self.handle, sys, C.c_void_p(v.data_ptr()),
                                    C.c_void_p(out.data_ptr()), v.shape[0], components))
        return out[0] if squeeze else out

    def tridiagonal(self, sys: int = 0):
        R, m = self.params.n_probes, self.params.n_steps
        a = (C.c_double * (R * m))()
        b = (C.c_double * (R * m))()
        me = (C.c_int32 * R)()
        L.check(self.lib.mbd_get_tridiagonal(self.handle, sys, a, b, me))
        at = torch.tensor(list(a), dtype=torch.float64).reshape(R, m)
        bt = torch.tensor(list(b), dtype=torch.float64).reshape(R, m)
        return at, bt, torch.tensor(list(me), dtype=torch.int32)

    def quadrature(self, sys: int = 0) -> torch.Tensor:
        R = self.params.n_probes
        q = (C.c_double * R)()
        L.check(self.lib.mbd_get_quadrature(self.handle, sys, q))
        return torch.tensor(list(q), dtype=torch.float64)

    def set_positions(self, pos: torch.Tensor, sys: int = 0):
        pos = pos.to(dtype=torch.float64, device="cuda").contiguous()
        self._pos_keep = pos
        L.check(self.lib.mbd_set_positions(self.handle, sys, C.c_void_p(pos.data_ptr())))

    def set_timing(self, on: bool = True):
        L.check(self.lib.mbd_set_timing(self.handle, 1 if on else 0))

    def stage_times(self):
        """{stage: (total_ms, launches)} since the last call."""
        n = len(L.STAGES)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        L.check(self.lib.mbd_get_stage_times(self.handle, ms, cnt))
        return {L.STAGES[i]: (ms[i], cnt[i]) for i in range(n)}

    def scs(self, sys: int = 0, n_freq: int = 15, freq_scale: float = 0.6, tol: float = 1e-10,
            max_iter: int = 1000, with_freq: bool = False, noalloc: bool = False):
        """Range-separated self-consistent screening of system `sys` at its current
        positions (mbd_scs, or mbd_scs_noalloc with noalloc=True). Returns (alpha, omega,
        r_vdw) screened, float64 on the GPU in the caller's atom order, plus alpha^SCS at
        the n_freq quadrature nodes [n_freq, N] when with_freq, and an info dict
        (iterations, max_rel_residual)."""
        n = self.systems[sys].n
        out = torch.empty(3, n, dtype=torch.float64, device="cuda")
        af = torch.empty(n_freq, n, dtype=torch.float64, device="cuda") if with_freq else None
        prm = L.MbdScsParams(n_freq, freq_scale, tol, max_iter)
        inf = L.MbdScsInfo()
        fn = self.lib.mbd_scs_noalloc if noalloc else self.lib.mbd_scs
        L.check(fn(self.handle, sys, C.byref(prm), C.c_void_p(out[0].data_ptr()),
                   C.c_void_p(out[1].data_ptr()), C.c_void_p(out[2].data_ptr()),
                   C.c_void_p(af.data_ptr()) if with_freq else None, C.byref(inf)))
        info = {"iterations": inf.iterations, "max_rel_residual": inf.max_rel_residual}
        res = (out[0], out[1], out[2])
        return res + ((af,) if with_freq else ()) + (info,)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.mbd_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def energy(systems: List[DeviceSystem], params: Params) -> torch.Tensor:
    """E_MBD per system (float64 tensor on the GPU)."""
    plan = Plan(systems, params)
    try:
        e = plan.execute()
        plan.check()
        return e
    finally:
        plan.close()


class MBDEnergy(torch.autograd.Function):
    """E_MBD of one system as a differentiable function of its positions.

    forward(pos, plan) sets the positions, runs the plan with forces and returns the
    energy; backward returns grad_E * dE/dR = -grad_E * F. The plan must have been
    created with want_forces=True for this system (index 0)."""

    @staticmethod
    def forward(ctx, pos, plan):
        plan.set_positions(pos.detach())
        e, f = plan.execute(forces=True)
        plan.check()
        ctx.save_for_backward(f)
        return e[0]

    @staticmethod
    def backward(ctx, grad):
        (f,) = ctx.saved_tensors
        return -grad * f.to(grad.device), None
