"""Python binding of libvms: device buffers from PyTorch, every step in HIP.

The functions here only marshal arguments: they allocate tensors for the
C ABI (include/vms.h), pass their device pointers and the current torch
stream, and turn status codes into exceptions.  No part of the Newton step
runs in Python; if libvms.so is missing, or no HIP device is present, the
calls raise.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

VMS_OK, VMS_NOT_CONVERGED = 0, 1
ASM_RESIDUAL, ASM_TANGENT, ASM_RKCORR = 1, 2, 4
OP_FULL, OP_A, OP_B, OP_C, OP_D = 0, 1, 2, 3, 4
PC_LDU, PC_UPPER, PC_LOWER, PC_DIAG, PC_SIMPLE = 0, 1, 2, 3, 4
FP64, MIXED = 0, 1
ORTH_CGS2, ORTH_MGS, ORTH_CGS1, ORTH_CGS_IFNEEDED = 0, 1, 2, 3
AK_GMRES, AK_CG_INNER, AK_CG = 0, 1, 2
SHAT_CHEBYSHEV, SHAT_CG, SHAT_NONE = 0, 1, 2
SCHUR_KRYLOV, SCHUR_SHAT = 0, 1
APC_BJ, APC_AMG = 0, 1

STATE_KEYS = ("u_n", "p_n", "v_n", "du_n", "dp_n", "dv_n", "u", "p", "v", "du", "dp", "dv")


class VmsError(RuntimeError):
    def __init__(self, what, code, msg):
        super().__init__(f"{what}: status {code}: {msg}")
        self.code = code


def solver_opts(rtol=1e-8, atol=1e-50, maxit=200, rtol_A=5e-5, atol_A=1e-50, maxit_A=500,
                rtol_S=1.5e-5, atol_S=1e-50, maxit_S=200, rtol_I=7e-5, atol_I=1e-50, maxit_I=500,
                precond=PC_LDU, precision=FP64, orth=ORTH_CGS1, shat_degree=16,
                shat_ratio=20.0, a_krylov=AK_GMRES, cg_symmetrise=1, shat_method=SHAT_CG,
                schur_solve=SCHUR_KRYLOV, relax_inner=0, schur_mass=0.0, a_prec=APC_BJ) -> L.SolverOpts:
    return L.SolverOpts(rtol, atol, maxit, rtol_A, atol_A, maxit_A, rtol_S, atol_S, maxit_S,
                        rtol_I, atol_I, maxit_I, precond, precision, orth, shat_degree, shat_ratio, a_krylov,
                        cg_symmetrise, shat_method, schur_solve, relax_inner, schur_mass, a_prec, 0)


def amg_opts(max_levels=3, min_coarse=64, degree=2, coarse_degree=2, mid_degree=0) -> L.AmgOpts:
    return L.AmgOpts(max_levels, min_coarse, degree, coarse_degree, mid_degree)


def newton_opts(tol_R=1e-8, tol_A=1e-50, l_max=20, rk_corr=1, eps_diag=1e-15, dir_lift=0) -> L.NewtonOpts:
    return L.NewtonOpts(tol_R, tol_A, l_max, rk_corr, eps_diag, dir_lift, 0)


def time_int(dt, rho_inf=0.5, t_n=0.0, t_load=0.0) -> L.TimeInt:
    return L.TimeInt(dt, rho_inf, t_n, t_load)


def _p(t):
    return None if t is None else t.data_ptr()


@dataclass
class Matrix:
    A: torch.Tensor
    B: torch.Tensor
    C: torch.Tensor
    D: torch.Tensor
    W: torch.Tensor
    A32: torch.Tensor | None = None
    B32: torch.Tensor | None = None
    C32: torch.Tensor | None = None
    D32: torch.Tensor | None = None

    def c(self) -> L.Matrix:
        return L.Matrix(_p(self.A), _p(self.B), _p(self.C), _p(self.D), _p(self.A32), _p(self.B32),
                        _p(self.C32), _p(self.D32), _p(self.W))


class Problem:
    """One mesh + material on one device: pattern, contribution lists, dead load, context."""

    def __init__(self, mesh, mat, device="cuda:0", compact_shat=True):
        self.lib = L.load()
        self.dev = torch.device(device)
        if self.dev.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("libvms needs a HIP device (torch.cuda is not available)")
        lib = self.lib
        self.mesh = mesh
        n, m, f = mesh.n_nodes, mesh.n_tets, int(mesh.bfaces.shape[0])
        tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
        bfaces = np.ascontiguousarray(mesh.bfaces, dtype=np.int32).reshape(-1, 3)
        nnzb, sw, w2, span = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
        self._check(lib.vms_setup_sizes(n, m, tets.ctypes.data, C.byref(nnzb), C.byref(sw), C.byref(w2),
                                        C.byref(span)), "vms_setup_sizes", ctx=False)
        nz = nnzb.value
        self.shat_span = span.value
        compact = compact_shat and span.value <= 32767   # 2-byte S^ column offsets
        h = {"row_len": np.zeros(n, np.int32), "col": np.zeros(nz, np.int32), "tpos": np.zeros(nz, np.int32),
             "diag_pos": np.zeros(n, np.int32), "blk_src_ptr": np.zeros(nz + 1, np.int32),
             "blk_src": np.zeros(max(16 * m, 1), np.int32),
             "shat_col": np.zeros(n * w2.value, np.int32),
             "shat_off": np.zeros(n * w2.value if compact else 1, np.int16),
             "nf_ptr": np.zeros(n + 1, np.int32), "nf_face": np.zeros(max(3 * f, 1), np.int32)}
        ptrs = [h[k].ctypes.data for k in ("row_len", "col", "tpos", "diag_pos", "blk_src_ptr", "blk_src",
                                            "shat_col")]
        ptrs += [h["shat_off"].ctypes.data if compact else None, h["nf_ptr"].ctypes.data, h["nf_face"].ctypes.data]
        self._check(lib.vms_setup_build(n, m, tets.ctypes.data, f, bfaces.ctypes.data if f else None, *ptrs),
                    "vms_setup_build", ctx=False)
        self.slot_width = sw.value
        self.shat_width = w2.value
        h["row_ptr"] = (self.slot_width * np.arange(n + 1)).astype(np.int64)   # slot start of each row
        self.host = h
        self.nnzb = nz
        dev = self.dev

        def up(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)

        self.d = {"X": up(mesh.X, np.float64), "tets": up(tets, np.int32),
                  "bfaces": up(bfaces if f else np.zeros((1, 3)), np.int32),
                  "traction": up(mesh.traction if f else np.zeros((1, 3)), np.float64),
                  "dir_mask": up(mesh.dir_mask, np.uint8), "dir_vel": up(mesh.dir_vel, np.float64),
                  "fibre": up(mesh.fibre, np.float64) if mesh.fibre is not None else None}
        for k in ("col", "tpos", "diag_pos", "blk_src_ptr", "blk_src", "shat_col", "nf_ptr", "nf_face"):
            self.d[k] = up(h[k], np.int32)
        self.d["shat_off"] = up(h["shat_off"], np.int16) if compact else None
        d = self.d
        self.cmesh = L.Mesh(n, m, f, self.slot_width, nz, _p(d["X"]), _p(d["tets"]), _p(d["bfaces"]),
                            _p(d["traction"]), _p(d["dir_mask"]), _p(d["dir_vel"]), _p(d["fibre"]),
                            _p(d["col"]), _p(d["tpos"]), _p(d["diag_pos"]), _p(d["blk_src_ptr"]),
                            _p(d["blk_src"]), self.shat_width, _p(d["shat_col"]), _p(d["shat_off"]),
                            _p(d["nf_ptr"]), _p(d["nf_face"]), None)
        self.set_material(mat)
        self.stream = torch.cuda.current_stream(dev)
        ctx = C.c_void_p()
        rc = lib.vms_ctx_create(C.byref(ctx), dev.index or 0, C.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise VmsError("vms_ctx_create", rc, "no usable HIP device")
        self.ctx = ctx
        self.dfibre = None
        self.f_ext = torch.zeros(3 * n, dtype=torch.float64, device=dev)
        self._check(lib.vms_nodal_load(self.ctx, C.byref(self.cmesh), _p(self.f_ext)), "vms_nodal_load")
        self._ws = None
        self.amg = None

    def setup_amg(self, opts=None):
        """Build the multigrid hierarchy of the mesh (vms_amg_create, host), upload its fixed arrays
        into a device buffer (vms_amg_upload) and attach it to the mesh (a_prec = APC_AMG)."""
        lib, n = self.lib, self.mesh.n_nodes
        opts = opts or amg_opts()
        X = np.ascontiguousarray(self.mesh.X, dtype=np.float64)
        dm = np.ascontiguousarray(self.mesh.dir_mask, dtype=np.uint8)
        obj = C.c_void_p()
        self._check(lib.vms_amg_create(n, self.slot_width, self.host["row_len"].ctypes.data,
                                       self.host["col"].ctypes.data, X.ctypes.data, dm.ctypes.data,
                                       C.byref(opts), C.byref(obj)), "vms_amg_create", ctx=False)
        self.free_amg()
        self.amg = obj
        nb = lib.vms_amg_device_bytes(obj)
        self._amg_buf = torch.empty(int(nb), dtype=torch.uint8, device=self.dev)
        self._check(lib.vms_amg_upload(self.ctx, obj, _p(self._amg_buf), int(nb)), "vms_amg_upload")
        self.cmesh.amg = obj.value
        return self.amg_info()

    def amg_info(self):
        info = L.AmgInfo()
        self._check(self.lib.vms_amg_get_info(self.amg, C.byref(info)), "vms_amg_get_info", ctx=False)
        k = info.n_levels
        return {"n_levels": k, "n": list(info.n[:k]), "bs": list(info.bs[:k]), "nnzb": list(info.nnzb[:k]),
                "device_bytes": int(info.device_bytes)}

    def amg_level(self, level):
        """Host views of one level (copies): agg, P [n][bs][10], and for level >= 1 ptr, col, dropped."""
        info = self.amg_info()
        n, bs = info["n"][level], info["bs"][level]
        ptrs = [C.c_void_p() for _ in range(5)]
        self._check(self.lib.vms_amg_level_arrays(self.amg, level, *(C.byref(p) for p in ptrs)), "vms_amg_level_arrays",
                    ctx=False)
        out = {}
        if ptrs[0].value:
            out["agg"] = np.ctypeslib.as_array(C.cast(ptrs[0], C.POINTER(C.c_int32)), (n,)).copy()
            out["P"] = np.ctypeslib.as_array(C.cast(ptrs[1], C.POINTER(C.c_double)), (n * bs * 10,)).reshape(n, bs, 10).copy()
        if level > 0:
            nnzb = info["nnzb"][level]
            out["ptr"] = np.ctypeslib.as_array(C.cast(ptrs[2], C.POINTER(C.c_int32)), (n + 1,)).copy()
            out["col"] = np.ctypeslib.as_array(C.cast(ptrs[3], C.POINTER(C.c_int32)), (nnzb,)).copy()
            out["dropped"] = np.ctypeslib.as_array(C.cast(ptrs[4], C.POINTER(C.c_uint8)), (n * 10,)).copy()
        return out

    def amg_apply(self, K, r, sym=0):
        """z = one V-cycle for the scaled A of K (vms_amg_apply); r: [n][3] FP64 device tensor."""
        nb = self.lib.vms_amg_apply_workspace(C.byref(self.cmesh), sym)
        ws = self.workspace(nb + 512)
        z = torch.empty_like(r)
        self._check(self.lib.vms_amg_apply(self.ctx, C.byref(self.cmesh), C.byref(K.c()), sym, _p(r), _p(z), _p(ws),
                                           ws.numel()), "vms_amg_apply")
        return z

    def free_amg(self):
        if self.amg is not None:
            self.cmesh.amg = None
            self.lib.vms_amg_destroy(self.amg)
            self.amg = None

    # ---- helpers -----------------------------------------------------------
    def set_material(self, mat):
        kappa = float(mat.kappa) if np.isfinite(mat.kappa) else 0.0
        self.mat = mat
        self.cmat = L.Material(int(mat.kind), mat.rho0, mat.mu, kappa, mat.k1, mat.k2, mat.kd, mat.c_m)

    def _check(self, rc, what, ctx=True, allow_nc=False):
        if rc == 0 or (allow_nc and rc == VMS_NOT_CONVERGED):
            return rc
        msg = self.lib.vms_last_error(self.ctx).decode() if ctx else ""
        raise VmsError(what, rc, msg)

    def __del__(self):
        try:
            if getattr(self, "amg", None) is not None:
                self.free_amg()
            if getattr(self, "ctx", None):
                self.lib.vms_ctx_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def set_timing(self, enable):
        """Event-time every launch of the A-block product (vms_ctx_set_timing)."""
        self._check(self.lib.vms_ctx_set_timing(self.ctx, 1 if enable else 0), "vms_ctx_set_timing")

    def kernel_time(self, fp32=False):
        """(total ms, launches) of the A-block product since the last call (vms_ctx_kernel_time)."""
        ms, cnt = C.c_double(), C.c_int64()
        self._check(self.lib.vms_ctx_kernel_time(self.ctx, 1 if fp32 else 0, C.byref(ms), C.byref(cnt)),
                    "vms_ctx_kernel_time")
        return ms.value, cnt.value

    def workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.dev)
        return self._ws

    def new_state(self, init=None):
        """Device state; ``init`` maps any of u, p, v, du, dp, dv (numpy) to y_n."""
        n = self.mesh.n_nodes
        st = {}
        for k in STATE_KEYS:
            base = k[:-2] if k.endswith("_n") else k
            shape = (n,) if base in ("p", "dp") else (n, 3)
            st[k] = torch.zeros(shape, dtype=torch.float64, device=self.dev)
        if init:
            for k, v in init.items():
                st[k + "_n"].copy_(torch.from_numpy(np.asarray(v, dtype=np.float64)))
                st[k].copy_(torch.from_numpy(np.asarray(v, dtype=np.float64)))
        return st

    @staticmethod
    def cstate(st):
        return L.State(*(_p(st[k]) for k in STATE_KEYS))

    @staticmethod
    def roll(st):
        """y_n <- y_{n+1} after a converged step."""
        for k in ("u", "p", "v", "du", "dp", "dv"):
            st[k + "_n"].copy_(st[k])

    def new_matrix(self, mirror32=False) -> Matrix:
        nz, n, dev = self.nnzb, self.mesh.n_nodes, self.dev
        f64 = dict(dtype=torch.float64, device=dev)
        f32 = dict(dtype=torch.float32, device=dev)
        K = Matrix(torch.zeros(9, nz, **f64), torch.zeros(3, nz, **f64), torch.zeros(3, nz, **f64),
                   torch.zeros(nz, **f64), torch.ones(n, 4, **f64))
        if mirror32:
            K.A32, K.B32 = torch.zeros(9, nz, **f32), torch.zeros(3, nz, **f32)
            K.C32, K.D32 = torch.zeros(3, nz, **f32), torch.zeros(nz, **f32)
        return K

    # ---- entry points ----------------------------------------------------------
    def predictor(self, st, ti, dir_lift=0):
        self._check(self.lib.vms_predictor(self.ctx, C.byref(self.cmesh), C.byref(ti), C.byref(self.cstate(st)),
                                           dir_lift), "vms_predictor")

    def assemble(self, st, ti, flags, K=None, R=None, corr=None, load=True):
        n = self.mesh.n_nodes
        if flags & ASM_RESIDUAL and R is None:
            R = torch.empty(n, 4, dtype=torch.float64, device=self.dev)
        if flags & ASM_RKCORR and corr is None:
            corr = torch.empty(n, 4, dtype=torch.float64, device=self.dev)
        if flags & ASM_TANGENT and K is None:
            K = self.new_matrix()
        cK = K.c() if K is not None else L.Matrix()
        ws = self.workspace(self.lib.vms_assemble_workspace(C.byref(self.cmesh), flags) + 512)
        self._check(self.lib.vms_assemble(self.ctx, C.byref(self.cmesh), C.byref(self.cmat), C.byref(ti),
                                          C.byref(self.cstate(st)), _p(self.f_ext) if load else None,
                                          C.byref(cK), _p(R), _p(corr), flags, _p(ws), ws.numel()), "vms_assemble")
        return K, R, corr

    def residual_norm(self, st, ti, R):
        out = C.c_double()
        self._check(self.lib.vms_residual_norm(self.ctx, C.byref(self.cmesh), C.byref(ti), C.byref(self.cstate(st)),
                                               _p(R), C.byref(out)), "vms_residual_norm")
        return out.value

    def prepare(self, K, R, corr=None, eps_diag=1e-15, mirror32=False):
        rhs = torch.empty(self.mesh.n_nodes, 4, dtype=torch.float64, device=self.dev)
        self._check(self.lib.vms_prepare_system(self.ctx, C.byref(self.cmesh), C.byref(K.c()), _p(R), _p(corr),
                                                _p(rhs), eps_diag, 1 if mirror32 else 0), "vms_prepare_system")
        return rhs

    def spmv(self, K, op, x, fp32=False):
        n = self.mesh.n_nodes
        shape = {OP_FULL: (n, 4), OP_A: (n, 3), OP_B: (n, 3), OP_C: (n,), OP_D: (n,)}[op]
        y = torch.empty(shape, dtype=torch.float32 if fp32 else torch.float64, device=self.dev)
        self._check(self.lib.vms_spmv(self.ctx, C.byref(self.cmesh), C.byref(K.c()), op, _p(x), _p(y),
                                      1 if fp32 else 0), "vms_spmv")
        return y

    def schur_hat(self, K):
        """S^ of the scaled blocks of K: (off-diagonal [n][W2] on shat_col, diagonal, diag(S^)^-1)."""
        n = self.mesh.n_nodes
        S = torch.empty(n, self.shat_width, dtype=torch.float64, device=self.dev)
        Sd = torch.empty(n, dtype=torch.float64, device=self.dev)
        sdinv = torch.empty(n, dtype=torch.float64, device=self.dev)
        self._check(self.lib.vms_schur_hat(self.ctx, C.byref(self.cmesh), C.byref(K.c()), _p(S), _p(Sd), _p(sdinv)),
                    "vms_schur_hat")
        return S, Sd, sdinv

    def shat_spmv(self, S, Sd, x, out=None):
        """y = S^ x for (S, Sd) from schur_hat (FP64, or all FP32)."""
        fp32 = S.dtype == torch.float32
        for t in (S, Sd, x):
            if t.dtype != S.dtype or not t.is_contiguous() or t.device != self.dev:
                raise ValueError("shat_spmv: S, Sd, x must be contiguous, on the problem's device, one dtype")
        y = torch.empty_like(x) if out is None else out
        self._check(self.lib.vms_shat_spmv(self.ctx, C.byref(self.cmesh), _p(S), _p(Sd), _p(x), _p(y),
                                           1 if fp32 else 0), "vms_shat_spmv")
        return y

    def solve_scaled(self, K, rhs, opts, x=None, allow_nc=False):
        nb = self.lib.vms_solve_workspace(C.byref(self.cmesh), C.byref(opts))
        ws = self.workspace(nb + 512)
        if x is None:
            x = torch.empty_like(rhs)
        stats = L.SolveStats()
        self._check(self.lib.vms_solve_scaled(self.ctx, C.byref(self.cmesh), C.byref(K.c()), _p(rhs), _p(x),
                                              C.byref(opts), _p(ws), ws.numel(), C.byref(stats)),
                    "vms_solve_scaled", allow_nc=allow_nc)
        return x, stats.as_dict()

    def solve(self, K, R, opts, corr=None, eps_diag=1e-15, delta=None, allow_nc=False):
        """solve(K, R) -> Delta (vms_solve): K as assembled (overwritten with W K W, K.W written)."""
        nb = self.lib.vms_solve_workspace(C.byref(self.cmesh), C.byref(opts))
        ws = self.workspace(nb)
        if delta is None:
            delta = torch.empty_like(R)
        stats = L.SolveStats()
        self._check(self.lib.vms_solve(self.ctx, C.byref(self.cmesh), C.byref(K.c()), _p(R), _p(corr), _p(delta),
                                       eps_diag, C.byref(opts), _p(ws), ws.numel(), C.byref(stats)),
                    "vms_solve", allow_nc=allow_nc)
        return delta, stats.as_dict()

    def newton_update(self, st, ti, K, x, dir_lift=0):
        """Stage 2 and the update from x = x* (with K.W) or, for K = None, from x = Delta."""
        self._check(self.lib.vms_newton_update(self.ctx, C.byref(self.cmesh), C.byref(ti), C.byref(self.cstate(st)),
                                               _p(K.W) if K is not None else None, _p(x), dir_lift),
                    "vms_newton_update")

    def solve_transpose(self, K, Kt, g, opts, eps_diag=1e-15, lam=None, allow_nc=False):
        """K^T lam = g (vms_solve_transpose): K as assembled (overwritten with W K W, K.W written)."""
        nb = self.lib.vms_solve_workspace(C.byref(self.cmesh), C.byref(opts))
        ws = self.workspace(nb)
        if lam is None:
            lam = torch.empty_like(g)
        stats = L.SolveStats()
        self._check(self.lib.vms_solve_transpose(self.ctx, C.byref(self.cmesh), C.byref(K.c()), C.byref(Kt.c()),
                                                 _p(g), _p(lam), eps_diag, C.byref(opts), _p(ws), ws.numel(),
                                                 C.byref(stats)), "vms_solve_transpose", allow_nc=allow_nc)
        return lam, stats.as_dict()

    def solve_transpose_scaled(self, K, Kt, rhs, opts, x=None, allow_nc=False):
        nb = self.lib.vms_solve_workspace(C.byref(self.cmesh), C.byref(opts))
        ws = self.workspace(nb + 512)
        if x is None:
            x = torch.empty_like(rhs)
        stats = L.SolveStats()
        self._check(self.lib.vms_solve_transpose_scaled(self.ctx, C.byref(self.cmesh), C.byref(K.c()),
                                                        C.byref(Kt.c()), _p(rhs), _p(x), C.byref(opts), _p(ws),
                                                        ws.numel(), C.byref(stats)),
                    "vms_solve_transpose_scaled", allow_nc=allow_nc)
        return x, stats.as_dict()

    def adjoint_workspace(self, opts):
        nb = self.lib.vms_adjoint_workspace(C.byref(self.cmesh), C.byref(opts))
        return self.workspace(nb + 512)

    def param_sensitivity(self, st, ti, lam, pmask, opts=None):
        ws = self.adjoint_workspace(opts or solver_opts())
        out = (C.c_double * 5)()
        self._check(self.lib.vms_param_sensitivity(self.ctx, C.byref(self.cmesh), C.byref(self.cmat), C.byref(ti),
                                                   C.byref(self.cstate(st)), _p(self.dfibre), _p(lam), pmask,
                                                   out, _p(ws), ws.numel()), "vms_param_sensitivity")
        return np.array(out[:])

    def adjoint_step(self, st, ti, K, Kt, ybar1, ydbar1, pmask, dJ, opts, eps_diag=1e-15):
        """One backward step; returns (ybar0, ydbar0, stats) and updates dJ (numpy, 5) in place."""
        ws = self.adjoint_workspace(opts)
        ybar0 = torch.empty_like(ybar1)
        ydbar0 = torch.empty_like(ydbar1)
        acc = (C.c_double * 5)(*dJ)
        stats = L.SolveStats()
        self._check(self.lib.vms_adjoint_step(self.ctx, C.byref(self.cmesh), C.byref(self.cmat), C.byref(ti),
                                              C.byref(self.cstate(st)), _p(self.dfibre), C.byref(K.c()),
                                              C.byref(Kt.c()), _p(ybar1), _p(ydbar1), _p(ybar0), _p(ydbar0),
                                              pmask, acc, C.byref(opts), eps_diag, _p(ws), ws.numel(),
                                              C.byref(stats)), "vms_adjoint_step")
        dJ[:] = np.array(acc[:])
        return ybar0, ydbar0, stats.as_dict()

    def set_fibres(self, fibre, dfibre):
        """Upload fibre directions and their derivative with respect to the fibre angle."""
        self.d["fibre"] = torch.from_numpy(np.ascontiguousarray(fibre, dtype=np.float64)).to(self.dev)
        self.dfibre = torch.from_numpy(np.ascontiguousarray(dfibre, dtype=np.float64)).to(self.dev)
        self.cmesh.fibre = _p(self.d["fibre"])

    def step_noalloc(self, st, ti, nopts, sopts, K=None, allow_nc=False):
        """One time step through vms_step_noalloc (the library's static device scratch as workspace)."""
        if K is None:
            K = self.new_matrix(mirror32=(sopts.precision == MIXED))
        stats = L.StepStats()
        self._check(self.lib.vms_step_noalloc(self.ctx, C.byref(self.cmesh), C.byref(self.cmat), C.byref(ti),
                                              C.byref(self.cstate(st)), _p(self.f_ext), C.byref(K.c()),
                                              C.byref(nopts), C.byref(sopts), C.byref(stats)),
                    "vms_step_noalloc", allow_nc=allow_nc)
        return stats.as_dict(), K

    def step(self, st, ti, nopts, sopts, K=None, allow_nc=False):
        if K is None:
            K = self.new_matrix(mirror32=(sopts.precision == MIXED))
        nb = self.lib.vms_step_workspace(C.byref(self.cmesh), C.byref(sopts))
        ws = self.workspace(nb + 512)
        stats = L.StepStats()
        self._check(self.lib.vms_step(self.ctx, C.byref(self.cmesh), C.byref(self.cmat), C.byref(ti),
                                      C.byref(self.cstate(st)), _p(self.f_ext), C.byref(K.c()), C.byref(nopts),
                                      C.byref(sopts), _p(ws), ws.numel(), C.byref(stats)),
                    "vms_step", allow_nc=allow_nc)
        return stats.as_dict(), K
