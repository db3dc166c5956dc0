"""Python binding of the C ABI (include/lgt.h) over torch device tensors.

Every function marshals arguments and calls the function of the same name in
liblgt.so; all arithmetic runs in the library's HIP kernels.  Fields are
contiguous complex128 CUDA/HIP tensors in the canonical layouts:
gauge-type (Lt, Lz, Ly, Lx, 4, 3, 3), spinor (Lt, Lz, Ly, Lx, 4, 3).  Work is
ordered on torch's current stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib
from ._lib import (LGT_FP64, LGT_MIXED_FP32, LGT_MIXED_BF16, LGT_OUT_FORCE, LGT_OUT_GRAD,  # noqa: F401
                   LGT_OUT_MOMENTUM, SolverParams, SolverStats)

_MODES = {"force": LGT_OUT_FORCE, "grad": LGT_OUT_GRAD, "momentum": LGT_OUT_MOMENTUM}
_PRECISIONS = {"fp64": LGT_FP64, "mixed_fp32": LGT_MIXED_FP32, "mixed_bf16": LGT_MIXED_BF16}


class LGTError(RuntimeError):
    def __init__(self, status: int, message: str, stats: Optional[dict] = None):
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.stats = stats


class LGTNotConverged(LGTError):
    pass


class LGTNonFinite(LGTError):
    pass


@dataclass
class Params:
    """Solver parameters (lgt_solver_params)."""
    precision: str = "fp64"
    tol: float = 1e-10
    max_iter: int = 20000
    reliable_delta: float = 0.0  # 0: the library's default for the precision
    even_odd: int = 1
    first_pass_factor: float = 0.0  # 0: the library's default

    def to_c(self) -> SolverParams:
        return SolverParams(_PRECISIONS[self.precision], self.even_odd, float(self.tol),
                            int(self.max_iter), float(self.reliable_delta), float(self.first_pass_factor))


def _check(lib, ctx, status: int, stats: Optional[SolverStats] = None):
    if status == _lib.LGT_OK:
        return
    msg = lib.lgt_last_error(ctx)
    msg = msg.decode() if msg else ""
    st = stats.as_dict() if stats is not None else None
    if status == _lib.LGT_ERR_NOT_CONVERGED:
        raise LGTNotConverged(status, msg, st)
    if status == _lib.LGT_ERR_NONFINITE:
        raise LGTNonFinite(status, msg, st)
    raise LGTError(status, msg, st)


def _stream_ptr() -> int:
    return torch.cuda.current_stream().cuda_stream


class Batch:
    """A batch object (lgt_batch): batched solves whose items may sit on
    several lattices (one Lattice each)."""

    def __init__(self):
        self.lib = _lib.load()
        b = ctypes.c_void_p()
        st = self.lib.lgt_batch_create(ctypes.c_void_p(_stream_ptr()), ctypes.byref(b))
        if st != _lib.LGT_OK:
            raise LGTError(st, "lgt_batch_create failed", None)
        self.handle = b

    def close(self):
        if getattr(self, "handle", None):
            self.lib.lgt_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cg_solve(self, items, params: Optional["Params"] = None, want_y: bool = True):
        """lgt_cg_solve_batch over items [(lattice, U, phi, kappa), ...].
        Returns (Xs, Ys, stats) in item order."""
        params = params or Params()
        n = len(items)
        Xs = [lat.empty_spinor() for lat, _, _, _ in items]
        Ys = [lat.empty_spinor() for lat, _, _, _ in items] if want_y else [None] * n
        arr = (_lib.BatchItem * max(n, 1))()
        for k, (lat, U, phi, kappa) in enumerate(items):
            arr[k].ctx = lat.ctx
            arr[k].U = lat._field(U, "gauge", f"U[{k}]")
            arr[k].phi = lat._field(phi, "spinor", f"phi[{k}]")
            arr[k].X = lat._field(Xs[k], "spinor", f"X[{k}]")
            arr[k].Y_or_null = lat._field(Ys[k], "spinor", f"Y[{k}]") if want_y else None
            arr[k].kappa = float(kappa)
        stats = (SolverStats * max(n, 1))()
        cp = params.to_c()
        self.lib.lgt_batch_set_stream(self.handle, ctypes.c_void_p(_stream_ptr()))
        st = self.lib.lgt_cg_solve_batch(self.handle, n, arr, ctypes.byref(cp), stats)
        if st != _lib.LGT_OK:
            msg = self.lib.lgt_batch_last_error(self.handle)
            msg = msg.decode() if msg else ""
            s0 = stats[0].as_dict() if n else None
            if st == _lib.LGT_ERR_NOT_CONVERGED:
                raise LGTNotConverged(st, msg, s0)
            if st == _lib.LGT_ERR_NONFINITE:
                raise LGTNonFinite(st, msg, s0)
            raise LGTError(st, msg, s0)
        return Xs, Ys, [stats[k].as_dict() for k in range(n)]


class Lattice:
    """A library context (lgt_ctx) for one lattice geometry on the current device."""

    def __init__(self, dims, fermion_bc: int = -1):
        self.lib = _lib.load()
        self.dims = tuple(int(d) for d in dims)
        lx, ly, lz, lt = self.dims
        self.site_shape = (lt, lz, ly, lx)
        self.volume = lx * ly * lz * lt
        self.fermion_bc = int(fermion_bc)
        geom = _lib.Geom((ctypes.c_int32 * 4)(*self.dims), self.fermion_bc)
        ctx = ctypes.c_void_p()
        status = self.lib.lgt_create(ctypes.byref(geom), ctypes.c_void_p(_stream_ptr()), ctypes.byref(ctx))
        _check(self.lib, None, status)
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.lgt_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- marshalling helpers --------------------------------------------------
    def _bind_stream(self):
        self.lib.lgt_set_stream(self.ctx, ctypes.c_void_p(_stream_ptr()))

    def _field(self, t: torch.Tensor, kind: str, name: str) -> ctypes.c_void_p:
        shape = self.site_shape + ((4, 3, 3) if kind == "gauge" else (4, 3))
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.complex128 or tuple(t.shape) != shape:
            raise ValueError(f"{name}: expected complex128 {shape}, got {t.dtype} {tuple(t.shape)}")
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return ctypes.c_void_p(t.data_ptr())

    def empty_gauge(self):
        return torch.empty(self.site_shape + (4, 3, 3), dtype=torch.complex128, device="cuda")

    def empty_spinor(self):
        return torch.empty(self.site_shape + (4, 3), dtype=torch.complex128, device="cuda")

    # -- the ABI ----------------------------------------------------------------
    def dslash(self, U, psi, kappa: float, dagger: bool = False, out=None):
        """lgt_dslash: D psi (or D^dag psi)."""
        out = self.empty_spinor() if out is None else out
        self._bind_stream()
        st = self.lib.lgt_dslash(self.ctx, self._field(U, "gauge", "U"), self._field(psi, "spinor", "psi"),
                                 self._field(out, "spinor", "out"), float(kappa), int(bool(dagger)))
        _check(self.lib, self.ctx, st)
        return out

    def cg_solve(self, U, phi, kappa: float, params: Optional[Params] = None, want_y: bool = True):
        """lgt_cg_solve: X = (D^dag D)^-1 phi, Y = D X.  Returns (X, Y, stats)."""
        params = params or Params()
        X = self.empty_spinor()
        Y = self.empty_spinor() if want_y else None
        stats = SolverStats()
        cp = params.to_c()
        self._bind_stream()
        st = self.lib.lgt_cg_solve(self.ctx, self._field(U, "gauge", "U"), self._field(phi, "spinor", "phi"),
                                   self._field(X, "spinor", "X"),
                                   self._field(Y, "spinor", "Y") if Y is not None else None,
                                   float(kappa), ctypes.byref(cp), ctypes.byref(stats))
        _check(self.lib, self.ctx, st, stats)
        return X, Y, stats.as_dict()

    def dslash_batch(self, U, psis, kappas, dagger: bool = False, precision: str = "fp64"):
        """lgt_dslash_batch: [D_k psi_k] (or D_k^dag) for up to 16 fields in one batched hop."""
        n = len(psis)
        if len(kappas) != n:
            raise ValueError("one kappa per field")
        outs = [self.empty_spinor() for _ in range(n)]
        ins = (ctypes.c_void_p * n)(*[self._field(p, "spinor", f"psi[{k}]").value for k, p in enumerate(psis)])
        outp = (ctypes.c_void_p * n)(*[self._field(o, "spinor", f"out[{k}]").value for k, o in enumerate(outs)])
        ks = (ctypes.c_double * n)(*[float(k) for k in kappas])
        self._bind_stream()
        st = self.lib.lgt_dslash_batch(self.ctx, self._field(U, "gauge", "U"), n, ins, outp, ks, int(bool(dagger)),
                                       _PRECISIONS[precision])
        _check(self.lib, self.ctx, st)
        return outs

    def cg_solve_batch(self, U, phis, kappas, params: Optional[Params] = None, want_y: bool = True):
        """lgt_cg_solve_batch with every item on this lattice: one solve per
        (phi_n, kappa_n) through shared launches.  Returns (Xs, Ys, stats)."""
        if len(kappas) != len(phis):
            raise ValueError("one kappa per right-hand side")
        if getattr(self, "_batch", None) is None:
            self._batch = Batch()
        return self._batch.cg_solve([(self, U, phi, k) for phi, k in zip(phis, kappas)], params, want_y)

    def action(self, U, phi, beta: float, kappa: float, params: Optional[Params] = None,
               gauge: bool = True, fermion: bool = True):
        """lgt_action: returns (S_G or None, S_F or None, stats)."""
        params = params or Params()
        sg = ctypes.c_double()
        sf = ctypes.c_double()
        stats = SolverStats()
        cp = params.to_c()
        self._bind_stream()
        st = self.lib.lgt_action(self.ctx, self._field(U, "gauge", "U"),
                                 self._field(phi, "spinor", "phi") if fermion else None,
                                 float(beta), float(kappa), ctypes.byref(cp),
                                 ctypes.byref(sg) if gauge else None,
                                 ctypes.byref(sf) if fermion else None, ctypes.byref(stats))
        _check(self.lib, self.ctx, st, stats)
        return (sg.value if gauge else None), (sf.value if fermion else None), stats.as_dict()

    def mean_plaquette(self, U) -> float:
        """<(1/3) Re tr P_mu,nu(x)> over the 6V plaquettes, from lgt_action's S_G at beta = 1."""
        sg, _, _ = self.action(U, None, 1.0, 0.0, gauge=True, fermion=False)
        return 1.0 - sg / (6.0 * self.volume)

    def fermion_force(self, U, phi, kappa: float, params: Optional[Params] = None, mode: str = "force",
                      dt: float = 0.0, out=None):
        """lgt_fermion_force: returns (out, stats)."""
        params = params or Params()
        out = self.empty_gauge() if out is None else out
        stats = SolverStats()
        cp = params.to_c()
        self._bind_stream()
        st = self.lib.lgt_fermion_force(self.ctx, self._field(U, "gauge", "U"), self._field(phi, "spinor", "phi"),
                                        float(kappa), ctypes.byref(cp), _MODES[mode], float(dt),
                                        self._field(out, "gauge", "out"), ctypes.byref(stats))
        _check(self.lib, self.ctx, st, stats)
        return out, stats.as_dict()

    def bilinear_force(self, U, a, b, kappa: float, coeff: float, mode: str = "force", dt: float = 0.0,
                       out=None):
        """lgt_bilinear_force: force/gradient of coeff * Re[a^dag D(U) b]."""
        out = self.empty_gauge() if out is None else out
        self._bind_stream()
        st = self.lib.lgt_bilinear_force(self.ctx, self._field(U, "gauge", "U"), self._field(a, "spinor", "a"),
                                         self._field(b, "spinor", "b"), float(kappa), float(coeff), _MODES[mode],
                                         float(dt), self._field(out, "gauge", "out"))
        _check(self.lib, self.ctx, st)
        return out

    def gauge_force(self, U, beta: float, mode: str = "force", dt: float = 0.0, out=None):
        """lgt_gauge_force."""
        out = self.empty_gauge() if out is None else out
        self._bind_stream()
        st = self.lib.lgt_gauge_force(self.ctx, self._field(U, "gauge", "U"), float(beta), _MODES[mode],
                                      float(dt), self._field(out, "gauge", "out"))
        _check(self.lib, self.ctx, st)
        return out

    def link_update(self, U, P, dt: float):
        """lgt_link_update: U <- reunit(exp(dt P) U) in place."""
        self._bind_stream()
        st = self.lib.lgt_link_update(self.ctx, self._field(U, "gauge", "U"), self._field(P, "gauge", "P"),
                                      float(dt))
        _check(self.lib, self.ctx, st)
        return U

    def momenta_from_normals(self, normals, out=None):
        """lgt_momenta_from_normals: P = i sum_a c_a T_a from float64 normals [...,4,8]."""
        shape = self.site_shape + (4, 8)
        if not isinstance(normals, torch.Tensor) or normals.dtype != torch.float64 or tuple(normals.shape) != shape \
                or not normals.is_cuda or not normals.is_contiguous():
            raise ValueError(f"normals: expected a contiguous float64 device tensor of shape {shape}")
        out = self.empty_gauge() if out is None else out
        self._bind_stream()
        st = self.lib.lgt_momenta_from_normals(self.ctx, ctypes.c_void_p(normals.data_ptr()),
                                               self._field(out, "gauge", "P"))
        _check(self.lib, self.ctx, st)
        return out

    def kinetic(self, P) -> float:
        """lgt_kinetic."""
        k = ctypes.c_double()
        self._bind_stream()
        st = self.lib.lgt_kinetic(self.ctx, self._field(P, "gauge", "P"), ctypes.byref(k))
        _check(self.lib, self.ctx, st)
        return k.value

    def md_step(self, U, P, phi, beta: float, kappa: float, dt: float, nsteps: int,
                params: Optional[Params] = None):
        """lgt_md_step: leapfrog trajectory in place; returns (dH, stats)."""
        params = params or Params()
        dh = ctypes.c_double()
        stats = SolverStats()
        cp = params.to_c()
        self._bind_stream()
        st = self.lib.lgt_md_step(self.ctx, self._field(U, "gauge", "U"), self._field(P, "gauge", "P"),
                                  self._field(phi, "spinor", "phi") if phi is not None else None,
                                  float(beta), float(kappa), float(dt), int(nsteps), ctypes.byref(cp),
                                  ctypes.byref(dh), ctypes.byref(stats))
        _check(self.lib, self.ctx, st, stats)
        return dh.value, stats.as_dict()

    def stout_smear(self, U, rho: float, nlevels: int, out=None):
        """lgt_stout_smear: stout^n(U)."""
        out = self.empty_gauge() if out is None else out
        self._bind_stream()
        st = self.lib.lgt_stout_smear(self.ctx, self._field(U, "gauge", "U"), self._field(out, "gauge", "out"),
                                      float(rho), int(nlevels))
        _check(self.lib, self.ctx, st)
        return out

    def stout_backprop(self, U, G_top, rho: float, nlevels: int, out=None):
        """lgt_stout_backprop: gradient at U of Re tr(G_top^dag stout^n(U))."""
        out = self.empty_gauge() if out is None else out
        self._bind_stream()
        st = self.lib.lgt_stout_backprop(self.ctx, self._field(U, "gauge", "U"),
                                         self._field(G_top, "gauge", "G_top"), float(rho), int(nlevels),
                                         self._field(out, "gauge", "out"))
        _check(self.lib, self.ctx, st)
        return out

    def smeared_force(self, U, phi, beta: float, kappa: float, rho: float, nlevels: int,
                      params: Optional[Params] = None, mode: str = "force", dt: float = 0.0, out=None):
        """lgt_smeared_force: returns (out, S_F, stats)."""
        params = params or Params()
        out = self.empty_gauge() if out is None else out
        sf = ctypes.c_double()
        stats = SolverStats()
        cp = params.to_c()
        self._bind_stream()
        st = self.lib.lgt_smeared_force(self.ctx, self._field(U, "gauge", "U"), self._field(phi, "spinor", "phi"),
                                        float(beta), float(kappa), float(rho), int(nlevels), ctypes.byref(cp),
                                        _MODES[mode], float(dt), self._field(out, "gauge", "out"),
                                        ctypes.byref(sf), ctypes.byref(stats))
        _check(self.lib, self.ctx, st, stats)
        return out, sf.value, stats.as_dict()

    def md_step_smeared(self, U, P, phi, beta: float, kappa: float, rho: float, nlevels: int, dt: float,
                        nsteps: int, params: Optional[Params] = None):
        """lgt_md_step_smeared: leapfrog with the stout-smeared action; returns (dH, stats)."""
        params = params or Params()
        dh = ctypes.c_double()
        stats = SolverStats()
        cp = params.to_c()
        self._bind_stream()
        st = self.lib.lgt_md_step_smeared(self.ctx, self._field(U, "gauge", "U"), self._field(P, "gauge", "P"),
                                          self._field(phi, "spinor", "phi") if phi is not None else None,
                                          float(beta), float(kappa), float(rho), int(nlevels), float(dt),
                                          int(nsteps), ctypes.byref(cp), ctypes.byref(dh), ctypes.byref(stats))
        _check(self.lib, self.ctx, st, stats)
        return dh.value, stats.as_dict()

    def md_step_sw(self, U, P, phi, beta: float, kappa: float, dt: float, nsteps: int, n_inner: int,
                   params: Optional[Params] = None, rho: float = 0.0, nlevels: int = 0):
        """lgt_md_step_sw: Sexton-Weingarten trajectory (gauge force on n_inner
        sub-steps), plain (nlevels = 0) or smeared action; returns (dH, stats)."""
        params = params or Params()
        dh = ctypes.c_double()
        stats = SolverStats()
        cp = params.to_c()
        self._bind_stream()
        st = self.lib.lgt_md_step_sw(self.ctx, self._field(U, "gauge", "U"), self._field(P, "gauge", "P"),
                                     self._field(phi, "spinor", "phi") if phi is not None else None,
                                     float(beta), float(kappa), float(rho), int(nlevels), float(dt), int(nsteps),
                                     int(n_inner), ctypes.byref(cp), ctypes.byref(dh), ctypes.byref(stats))
        _check(self.lib, self.ctx, st, stats)
        return dh.value, stats.as_dict()

    def schur_dslash(self, U, psi, kappa: float, dagger: bool = False, out=None):
        """lgt_schur_dslash: Mhat psi (or Mhat^dag psi) on the odd sites, even sites zero."""
        out = self.empty_spinor() if out is None else out
        self._bind_stream()
        st = self.lib.lgt_schur_dslash(self.ctx, self._field(U, "gauge", "U"), self._field(psi, "spinor", "psi"),
                                       self._field(out, "spinor", "out"), float(kappa), int(bool(dagger)))
        _check(self.lib, self.ctx, st)
        return out

    def fermion_force_eo(self, U, phi, kappa: float, params: Optional[Params] = None, mode: str = "force",
                         dt: float = 0.0, out=None):
        """lgt_fermion_force_eo: returns (out, S_eo, stats)."""
        params = params or Params()
        out = self.empty_gauge() if out is None else out
        sf = ctypes.c_double()
        stats = SolverStats()
        cp = params.to_c()
        self._bind_stream()
        st = self.lib.lgt_fermion_force_eo(self.ctx, self._field(U, "gauge", "U"), self._field(phi, "spinor", "phi"),
                                           float(kappa), ctypes.byref(cp), _MODES[mode], float(dt),
                                           self._field(out, "gauge", "out"), ctypes.byref(sf), ctypes.byref(stats))
        _check(self.lib, self.ctx, st, stats)
        return out, sf.value, stats.as_dict()

    def md_step_eo(self, U, P, phi, beta: float, kappa: float, dt: float, nsteps: int, n_inner: int = 1,
                   params: Optional[Params] = None):
        """lgt_md_step_eo: trajectory with the even/odd-preconditioned action; returns (dH, stats)."""
        params = params or Params()
        dh = ctypes.c_double()
        stats = SolverStats()
        cp = params.to_c()
        self._bind_stream()
        st = self.lib.lgt_md_step_eo(self.ctx, self._field(U, "gauge", "U"), self._field(P, "gauge", "P"),
                                     self._field(phi, "spinor", "phi") if phi is not None else None,
                                     float(beta), float(kappa), float(dt), int(nsteps), int(n_inner),
                                     ctypes.byref(cp), ctypes.byref(dh), ctypes.byref(stats))
        _check(self.lib, self.ctx, st, stats)
        return dh.value, stats.as_dict()

    def cg_solve_multishift(self, U, phi, kappa: float, shifts, params: Optional[Params] = None):
        """lgt_cg_solve_multishift: X_i = (Mhat^dag Mhat + shifts[i])^-1 phi_o for every shift.

        Returns (Xs, stats): one spinor per shift (zero on even sites)."""
        params = params or Params()
        n = len(shifts)
        Xs = [self.empty_spinor() for _ in range(n)]
        sh = (ctypes.c_double * max(n, 1))(*[float(v) for v in shifts])
        ptrs = (ctypes.c_void_p * max(n, 1))(*[self._field(x, "spinor", f"X[{i}]") for i, x in enumerate(Xs)])
        stats = SolverStats()
        cp = params.to_c()
        self._bind_stream()
        st = self.lib.lgt_cg_solve_multishift(self.ctx, self._field(U, "gauge", "U"),
                                              self._field(phi, "spinor", "phi"), float(kappa), n, sh, ptrs,
                                              ctypes.byref(cp), ctypes.byref(stats))
        _check(self.lib, self.ctx, st, stats)
        return Xs, stats.as_dict()

    def rational_force_eo(self, U, phi, kappa: float, shifts, residues, a0: float = 0.0,
                          params: Optional[Params] = None, mode: str = "force", dt: float = 0.0, out=None):
        """lgt_rational_force_eo: force of phi_o^dag [a0 + sum_i r_i (A + s_i)^-1] phi_o; returns (out, S_R, stats)."""
        params = params or Params()
        n = len(shifts)
        if len(residues) != n:
            raise ValueError("one residue per shift")
        out = self.empty_gauge() if out is None else out
        sh = (ctypes.c_double * max(n, 1))(*[float(v) for v in shifts])
        rs = (ctypes.c_double * max(n, 1))(*[float(v) for v in residues])
        sr = ctypes.c_double()
        stats = SolverStats()
        cp = params.to_c()
        self._bind_stream()
        st = self.lib.lgt_rational_force_eo(self.ctx, self._field(U, "gauge", "U"), self._field(phi, "spinor", "phi"),
                                            float(kappa), n, sh, rs, float(a0), ctypes.byref(cp), _MODES[mode],
                                            float(dt), self._field(out, "gauge", "out"), ctypes.byref(sr),
                                            ctypes.byref(stats))
        _check(self.lib, self.ctx, st, stats)
        return out, sr.value, stats.as_dict()

    def set_stout_checkpoints(self, max_stored_levels: int = -1):
        """lgt_set_stout_checkpoints: cap on the smearing levels kept for the reverse pass (-1: automatic)."""
        _check(self.lib, self.ctx, self.lib.lgt_set_stout_checkpoints(self.ctx, int(max_stored_levels)))

    def set_hop_block_sites(self, sites: int = 0):
        """lgt_set_hop_block_sites: sites per hop block, 32 or 64 (0: by volume)."""
        _check(self.lib, self.ctx, self.lib.lgt_set_hop_block_sites(self.ctx, int(sites)))

    def set_hop_block_order(self, order: int = 0):
        """lgt_set_hop_block_order: 64-site block order, 1 site order, 2 t-fastest (0: by volume)."""
        _check(self.lib, self.ctx, self.lib.lgt_set_hop_block_order(self.ctx, int(order)))

    def set_batch_hop_kernel(self, kind: str = "auto"):
        """lgt_set_batch_hop_kernel: FP32 batched hop kernel, "auto" (timed), "valu" or "mfma"."""
        code = {"auto": 0, "valu": 1, "mfma": 2}[kind]
        _check(self.lib, self.ctx, self.lib.lgt_set_batch_hop_kernel(self.ctx, code))

    def stout_last_schedule(self) -> dict:
        """lgt_stout_last_schedule: levels kept and passes recomputed by the last reverse pass."""
        s, p = ctypes.c_int32(), ctypes.c_int64()
        _check(self.lib, self.ctx, self.lib.lgt_stout_last_schedule(self.ctx, ctypes.byref(s), ctypes.byref(p)))
        return {"stored_levels": s.value, "recompute_passes": p.value}

    def hop_benchmark(self, U, psi, precision: str = "fp64", nrep: int = 50) -> float:
        """lgt_hop_benchmark: mean duration (ms) of one even/odd hop launch."""
        ms = ctypes.c_double()
        self._bind_stream()
        st = self.lib.lgt_hop_benchmark(self.ctx, self._field(U, "gauge", "U"), self._field(psi, "spinor", "psi"),
                                        _PRECISIONS[precision], int(nrep), ctypes.byref(ms))
        _check(self.lib, self.ctx, st)
        return ms.value

    def hop_benchmark_mrhs(self, U, psi, nrhs: int, precision: str = "mixed_fp32", nrep: int = 50) -> float:
        """lgt_hop_benchmark_mrhs: mean duration (ms) of one batched hop over nrhs fields."""
        ms = ctypes.c_double()
        self._bind_stream()
        st = self.lib.lgt_hop_benchmark_mrhs(self.ctx, self._field(U, "gauge", "U"),
                                             self._field(psi, "spinor", "psi"), int(nrhs),
                                             _PRECISIONS[precision], int(nrep), ctypes.byref(ms))
        _check(self.lib, self.ctx, st)
        return ms.value


# Module-level functions with the ABI's names.
def stout_schedule(nlevels: int, stored_levels: int) -> dict:
    """lgt_stout_schedule (host only): recomputed passes and forward checkpoints of the
    reverse pass through nlevels stout levels with stored_levels slots."""
    lib = _lib.load()
    passes = ctypes.c_int64()
    cp = (ctypes.c_int32 * max(1, int(stored_levels)))()
    ncp = ctypes.c_int32()
    st = lib.lgt_stout_schedule(int(nlevels), int(stored_levels), ctypes.byref(passes), cp, ctypes.byref(ncp))
    if st != _lib.LGT_OK:
        raise LGTError(st, "invalid schedule arguments")
    return {"recompute_passes": passes.value, "checkpoints": [cp[i] for i in range(ncp.value)]}


def lgt_dslash_noalloc(dims, U, psi, out, kappa: float, dagger: bool = False, fermion_bc: int = -1):
    """lgt_dslash_noalloc: D psi (or D^dag psi) into the caller's out, with
    no context and no device allocation (library-held scratch, V <= 16^4)."""
    lib = _lib.load()
    dims = tuple(int(d) for d in dims)
    lx, ly, lz, lt = dims
    shapes = {"U": (lt, lz, ly, lx, 4, 3, 3), "psi": (lt, lz, ly, lx, 4, 3), "out": (lt, lz, ly, lx, 4, 3)}
    for name, t in (("U", U), ("psi", psi), ("out", out)):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or tuple(t.shape) != shapes[name] \
                or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous complex128 device tensor of shape {shapes[name]}")
    geom = _lib.Geom((ctypes.c_int32 * 4)(*dims), int(fermion_bc))
    st = lib.lgt_dslash_noalloc(ctypes.byref(geom), ctypes.c_void_p(_stream_ptr()), ctypes.c_void_p(U.data_ptr()),
                                ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(out.data_ptr()), float(kappa),
                                int(bool(dagger)))
    _check(lib, None, st)
    return out


def lgt_create(dims, fermion_bc: int = -1) -> Lattice:
    return Lattice(dims, fermion_bc)


def lgt_dslash(lat: Lattice, U, psi, kappa, dagger=False, out=None):
    return lat.dslash(U, psi, kappa, dagger, out)


def lgt_cg_solve(lat: Lattice, U, phi, kappa, params=None, want_y=True):
    return lat.cg_solve(U, phi, kappa, params, want_y)


def lgt_cg_solve_batch(batch: Batch, items, params=None, want_y=True):
    return batch.cg_solve(items, params, want_y)


def lgt_action(lat: Lattice, U, phi, beta, kappa, params=None, gauge=True, fermion=True):
    return lat.action(U, phi, beta, kappa, params, gauge, fermion)


def lgt_fermion_force(lat: Lattice, U, phi, kappa, params=None, mode="force", dt=0.0, out=None):
    return lat.fermion_force(U, phi, kappa, params, mode, dt, out)


def lgt_bilinear_force(lat: Lattice, U, a, b, kappa, coeff, mode="force", dt=0.0, out=None):
    return lat.bilinear_force(U, a, b, kappa, coeff, mode, dt, out)


def lgt_gauge_force(lat: Lattice, U, beta, mode="force", dt=0.0, out=None):
    return lat.gauge_force(U, beta, mode, dt, out)


def lgt_link_update(lat: Lattice, U, P, dt):
    return lat.link_update(U, P, dt)


def lgt_kinetic(lat: Lattice, P):
    return lat.kinetic(P)


def lgt_md_step(lat: Lattice, U, P, phi, beta, kappa, dt, nsteps, params=None):
    return lat.md_step(U, P, phi, beta, kappa, dt, nsteps, params)


def lgt_hop_benchmark(lat: Lattice, U, psi, precision="fp64", nrep=50):
    return lat.hop_benchmark(U, psi, precision, nrep)


def lgt_hop_benchmark_mrhs(lat: Lattice, U, psi, nrhs, precision="mixed_fp32", nrep=50):
    return lat.hop_benchmark_mrhs(U, psi, nrhs, precision, nrep)


def lgt_stout_smear(lat: Lattice, U, rho, nlevels, out=None):
    return lat.stout_smear(U, rho, nlevels, out)


def lgt_stout_backprop(lat: Lattice, U, G_top, rho, nlevels, out=None):
    return lat.stout_backprop(U, G_top, rho, nlevels, out)


def lgt_smeared_force(lat: Lattice, U, phi, beta, kappa, rho, nlevels, params=None, mode="force", dt=0.0,
                      out=None):
    return lat.smeared_force(U, phi, beta, kappa, rho, nlevels, params, mode, dt, out)


def lgt_md_step_smeared(lat: Lattice, U, P, phi, beta, kappa, rho, nlevels, dt, nsteps, params=None):
    return lat.md_step_smeared(U, P, phi, beta, kappa, rho, nlevels, dt, nsteps, params)


def lgt_schur_dslash(lat: Lattice, U, psi, kappa, dagger=False, out=None):
    return lat.schur_dslash(U, psi, kappa, dagger, out)


def lgt_fermion_force_eo(lat: Lattice, U, phi, kappa, params=None, mode="force", dt=0.0, out=None):
    return lat.fermion_force_eo(U, phi, kappa, params, mode, dt, out)


def lgt_md_step_eo(lat: Lattice, U, P, phi, beta, kappa, dt, nsteps, n_inner=1, params=None):
    return lat.md_step_eo(U, P, phi, beta, kappa, dt, nsteps, n_inner, params)


def lgt_md_step_sw(lat: Lattice, U, P, phi, beta, kappa, rho, nlevels, dt, nsteps, n_inner, params=None):
    return lat.md_step_sw(U, P, phi, beta, kappa, dt, nsteps, n_inner, params, rho, nlevels)


def lgt_cg_solve_multishift(lat: Lattice, U, phi, kappa, shifts, params=None):
    return lat.cg_solve_multishift(U, phi, kappa, shifts, params)


def lgt_rational_force_eo(lat: Lattice, U, phi, kappa, shifts, residues, a0=0.0, params=None, mode="force", dt=0.0,
                          out=None):
    return lat.rational_force_eo(U, phi, kappa, shifts, residues, a0, params, mode, dt, out)
