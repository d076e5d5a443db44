"""ctypes binding of libvms.so (argument marshalling only).

Each function carries the name of the C entry point it calls and takes torch
tensors that already live on the GPU; every step of the method runs in the
library's HIP kernels.  The library must be built (paper_0809_4802_amd/build.py);
importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# VMS_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("VMS_LIBRARY", os.path.join(_PKG, "libvms.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_0809_4802_amd/build.py`")
_lib = ctypes.CDLL(LIB_PATH)

VMS_OK, VMS_EINVAL, VMS_EDEGENERATE, VMS_ESINGULAR_KFF = 0, -1, -2, -3
VMS_ENOCONV_GMRES, VMS_ENOCONV_NEWTON, VMS_ENONFINITE, VMS_EHIP, VMS_ENOMEM = -4, -5, -6, -7, -8
STATUS_NAMES = {0: "VMS_OK", -1: "VMS_EINVAL", -2: "VMS_EDEGENERATE", -3: "VMS_ESINGULAR_KFF",
                -4: "VMS_ENOCONV_GMRES", -5: "VMS_ENOCONV_NEWTON", -6: "VMS_ENONFINITE",
                -7: "VMS_EHIP", -8: "VMS_ENOMEM"}
VMS_FP64, VMS_MIXED = 0, 1
VMS_PC_BLOCK_JACOBI, VMS_PC_LEARNED = 0, 1
VMS_LIN_NEWTON, VMS_LIN_PICARD = 0, 1
PC_NIN, PC_NHID, PC_NOUT = 25, 64, 16
PC_NWEIGHTS = PC_NHID * PC_NIN + PC_NHID + PC_NOUT * PC_NHID + PC_NOUT

EXPORTED = ["vms_create", "vms_destroy", "vms_last_error", "vms_bsr_info", "vms_element_tangents",
            "vms_condense_assemble", "vms_condense_assemble_noalloc", "vms_residual", "vms_recover_update", "vms_bsr_spmv",
            "vms_gmres_solve", "vms_newton_step", "vms_full_info", "vms_full_assemble",
            "vms_full_newton_step", "vms_pc_features", "vms_pc_blocks",
            "vms_pc_train_step", "vms_profile", "vms_profile_read", "vms_set_linearization"]
PHASES = ["condense", "residual", "recover", "pc_setup", "pc_apply", "spmv", "dots", "update", "fill"]


class VmsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_elems", ctypes.c_int32),
                ("xyz", ctypes.c_void_p), ("tets", ctypes.c_void_p),
                ("n_dirichlet", ctypes.c_int32), ("dirichlet_dofs", ctypes.c_void_p)]


class CreateOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("max_restart", ctypes.c_int32), ("full_system", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("basis_fp64", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("pc", ctypes.c_int), ("pc_weights", ctypes.c_void_p), ("refine_max", ctypes.c_int32),
                ("inner_rtol", ctypes.c_double), ("cgs2", ctypes.c_int32),
                ("coarse_pressure", ctypes.c_int32), ("log_residuals", ctypes.c_void_p),
                ("log_max", ctypes.c_int32), ("deflate", ctypes.c_int32), ("basis_fp64", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("fell_back_to_bj", ctypes.c_int32), ("true_rel_res", ctypes.c_double),
                ("logged", ctypes.c_int32), ("singular_blocks", ctypes.c_int32),
                ("deflation_stopped", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NewtonOpts(ctypes.Structure):
    _fields_ = [("lin", SolveOpts)]


class NewtonInfo(ctypes.Structure):
    _fields_ = [("rnorm_before", ctypes.c_double), ("rnorm_after", ctypes.c_double), ("lin", SolveInfo),
                ("bad_elem", ctypes.c_int32)]


_vp = ctypes.c_void_p
_d = ctypes.c_double
_i32 = ctypes.c_int32
_sig = {
    "vms_create": [ctypes.POINTER(MeshDesc), ctypes.POINTER(CreateOpts), _vp, ctypes.POINTER(_vp)],
    "vms_destroy": [_vp],
    "vms_last_error": [_vp],
    "vms_bsr_info": [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                     ctypes.POINTER(_vp), ctypes.POINTER(_i32)],
    "vms_element_tangents": [_vp, _vp, _vp, _vp, _d, _d, _vp, _vp, _vp, _vp],
    "vms_condense_assemble": [_vp, _vp, _vp, _vp, _d, _d, _vp, _vp, _vp, _vp, _vp],
    "vms_condense_assemble_noalloc": [_vp, _vp, _vp, _vp, _d, _d, _vp, _vp, _vp, _vp, _vp],
    "vms_residual": [_vp, _vp, _vp, _vp, _d, _d, _vp, _vp, _vp, _vp],
    "vms_recover_update": [_vp, _vp, _vp, _vp, _d, _d, _vp, _vp, _vp],
    "vms_bsr_spmv": [_vp, _vp, _vp, _vp, _vp],
    "vms_gmres_solve": [_vp, _vp, _vp, _vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _vp],
    "vms_newton_step": [_vp, _vp, _vp, _vp, _d, _d, _vp, ctypes.POINTER(NewtonOpts),
                        ctypes.POINTER(NewtonInfo), _vp],
    "vms_set_linearization": [_vp, ctypes.c_int],
    "vms_full_info": [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_i32), ctypes.POINTER(_vp),
                      ctypes.POINTER(_vp)],
    "vms_full_assemble": [_vp, _vp, _vp, _vp, _d, _d, _vp, _vp, _vp, _vp, _vp],
    "vms_full_newton_step": [_vp, _vp, _vp, _vp, _d, _d, _vp, ctypes.POINTER(NewtonOpts),
                             ctypes.POINTER(NewtonInfo), _vp],
    "vms_pc_features": [_vp, _vp, _vp, _vp],
    "vms_pc_blocks": [_vp, _vp, _vp, _vp, _vp],
    "vms_pc_train_step": [_vp, _vp, _vp, _i32, _vp, _vp, _i32, ctypes.c_float, _vp, _vp, _vp],
    "vms_profile": [_vp, ctypes.c_uint32, ctypes.c_int32],
    "vms_profile_read": [_vp, _vp, _vp, _vp],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_char_p if _name == "vms_last_error" else ctypes.c_int


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc, ctx=None, allow=()):
    if rc != VMS_OK and rc not in allow:
        msg = _lib.vms_last_error(ctx)
        raise VmsError(rc, msg.decode() if msg else "")
    return rc


def _dev(t, dtype, shape=None):
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t


class Context:
    """Owns a vms_ctx*.  Tensors passed to it must be CUDA (HIP) tensors."""

    def __init__(self, xyz, tets, dirichlet_dofs, precision=VMS_FP64, max_restart=50, full_system=False,
                 stream=None, deterministic=False, basis_fp64=False):
        xyz = _dev(xyz, torch.float64).contiguous()
        tets = _dev(tets, torch.int32).contiguous()
        dd = _dev(dirichlet_dofs, torch.int32).contiguous()
        self.n_nodes = int(xyz.shape[0])
        self.n_elems = int(tets.shape[0])
        self.precision = precision
        self.dtype = torch.float64 if precision == VMS_FP64 else torch.float32
        desc = MeshDesc(self.n_nodes, self.n_elems, xyz.data_ptr(), tets.data_ptr(), int(dd.numel()),
                        dd.data_ptr() if dd.numel() else None)
        opts = CreateOpts(precision, max_restart, 1 if full_system else 0, 1 if deterministic else 0,
                          1 if basis_fp64 else 0)
        h = ctypes.c_void_p()
        _check(_lib.vms_create(ctypes.byref(desc), ctypes.byref(opts), _stream(stream), ctypes.byref(h)))
        self.handle = h
        nb = ctypes.c_int64()
        _check(_lib.vms_bsr_info(h, ctypes.byref(nb), None, None, None, None), h)
        self.nb = int(nb.value)
        self.device = xyz.device
        self.full_nb = self.full_rows = None
        if full_system:
            fnb, frows = ctypes.c_int64(), ctypes.c_int32()
            _check(_lib.vms_full_info(h, ctypes.byref(fnb), ctypes.byref(frows), None, None), h)
            self.full_nb, self.full_rows = int(fnb.value), int(frows.value)

    def close(self):
        if getattr(self, "handle", None):
            _lib.vms_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- allocation helpers (torch owns the memory) ------------------------------------
    def new_bsr(self):
        return torch.zeros((self.nb, 16), dtype=self.dtype, device=self.device)

    def new_vec(self, dtype=torch.float64):
        return torch.zeros((self.n_nodes, 4), dtype=dtype, device=self.device)

    def new_full_bsr(self):
        return torch.zeros((self.full_nb, 16), dtype=self.dtype, device=self.device)

    def new_full_vec(self):
        return torch.zeros((self.full_rows, 4), dtype=torch.float64, device=self.device)

    def full_pattern(self):
        """(rowptr, colidx) of the uncondensed system copied to host numpy arrays."""
        rp, ci = ctypes.c_void_p(), ctypes.c_void_p()
        _check(_lib.vms_full_info(self.handle, None, None, ctypes.byref(rp), ctypes.byref(ci)), self.handle)
        out = []
        for ptr, n in ((rp, self.full_rows + 1), (ci, self.full_nb)):
            t = torch.empty(n, dtype=torch.int32, device=self.device)
            torch.cuda.synchronize()
            _copy_device(t, ptr.value, n * 4)
            out.append(t.cpu().numpy())
        return tuple(out)

    def bsr_pattern(self):
        """(rowptr, colidx, diagpos) copied to host numpy arrays."""
        import numpy as np
        rp, ci, dp = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(_lib.vms_bsr_info(self.handle, None, ctypes.byref(rp), ctypes.byref(ci), ctypes.byref(dp),
                                 None), self.handle)
        out = []
        for ptr, n in ((rp, self.n_nodes + 1), (ci, self.nb), (dp, self.n_nodes)):
            t = torch.empty(n, dtype=torch.int32, device=self.device)
            torch.cuda.synchronize()
            _copy_device(t, ptr.value, n * 4)
            out.append(t.cpu().numpy())
        return tuple(out)


_hip = None


def _copy_device(dst, src_ptr, nbytes):
    """Device-to-device copy from a raw library pointer into a torch tensor."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
    hip = _hip
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    rc = hip.hipMemcpy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src_ptr), nbytes, 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")


def solve_opts(restart=50, max_iters=100000, rtol=1e-8, pc=VMS_PC_BLOCK_JACOBI, pc_weights=None,
               refine_max=30, inner_rtol=0.0, cgs2=1, coarse_pressure=1, log_residuals=None, deflate=0,
               basis_fp64=0):
    """log_residuals: device float tensor [k, n_nodes, 4] receiving restart residuals (or None).
    deflate: vectors kept by deflated restarting (0: plain restarts).  basis_fp64: on a mixed
    context (created with basis_fp64=True), an FP64 Krylov basis over the FP32-stored matrix
    and preconditioner."""
    return SolveOpts(restart, max_iters, rtol, pc,
                     pc_weights.data_ptr() if pc_weights is not None else None,
                     refine_max, inner_rtol, cgs2, coarse_pressure,
                     log_residuals.data_ptr() if log_residuals is not None else None,
                     int(log_residuals.shape[0]) if log_residuals is not None else 0, deflate, basis_fp64)


# ---- entry points (same names as the C ABI) ------------------------------------------
def vms_element_tangents(ctx: Context, u, beta, Re, dt=0.0, u_prev=None, body=None, Ke=None, Rvec=None,
                         stream=None):
    if Ke is None:
        Ke = torch.empty((ctx.n_elems, 19, 19), dtype=torch.float64, device=ctx.device)
    if Rvec is None:
        Rvec = torch.empty((ctx.n_elems, 19), dtype=torch.float64, device=ctx.device)
    _check(_lib.vms_element_tangents(ctx.handle, _ptr(u), _ptr(u_prev), _ptr(beta), float(Re), float(dt),
                                     _ptr(body), _ptr(Ke), _ptr(Rvec), _stream(stream)), ctx.handle)
    return Ke, Rvec


def vms_condense_assemble(ctx: Context, u, beta, Re, dt=0.0, u_prev=None, body=None, bsr_vals=None, rhs=None,
                          rnorm=None, stream=None):
    bsr_vals = ctx.new_bsr() if bsr_vals is None else bsr_vals
    rhs = ctx.new_vec() if rhs is None else rhs
    rnorm = torch.zeros(1, dtype=torch.float64, device=ctx.device) if rnorm is None else rnorm
    _check(_lib.vms_condense_assemble(ctx.handle, _ptr(u), _ptr(u_prev), _ptr(beta), float(Re), float(dt),
                                      _ptr(body), _ptr(bsr_vals), _ptr(rhs), _ptr(rnorm), _stream(stream)),
           ctx.handle)
    return bsr_vals, rhs, rnorm


def vms_condense_assemble_noalloc(ctx: Context, u, beta, Re, bsr_vals, rhs, rnorm, dt=0.0, u_prev=None, body=None,
                                  stream=None):
    """The no-allocation variant: every output buffer comes from the caller (nothing is allocated
    here either)."""
    _check(_lib.vms_condense_assemble_noalloc(ctx.handle, _ptr(u), _ptr(u_prev), _ptr(beta), float(Re), float(dt),
                                              _ptr(body), _ptr(bsr_vals), _ptr(rhs), _ptr(rnorm), _stream(stream)),
           ctx.handle)
    return bsr_vals, rhs, rnorm


def vms_residual(ctx: Context, u, beta, Re, dt=0.0, u_prev=None, body=None, rglob=None, rnorm=None,
                 stream=None):
    rglob = ctx.new_vec() if rglob is None else rglob
    rnorm = torch.zeros(1, dtype=torch.float64, device=ctx.device) if rnorm is None else rnorm
    _check(_lib.vms_residual(ctx.handle, _ptr(u), _ptr(u_prev), _ptr(beta), float(Re), float(dt), _ptr(body),
                             _ptr(rglob), _ptr(rnorm), _stream(stream)), ctx.handle)
    return rglob, rnorm


def vms_recover_update(ctx: Context, u, beta, du, Re, dt=0.0, u_prev=None, body=None, stream=None):
    _check(_lib.vms_recover_update(ctx.handle, _ptr(u), _ptr(beta), _ptr(u_prev), float(Re), float(dt),
                                   _ptr(body), _ptr(du), _stream(stream)), ctx.handle)


def vms_bsr_spmv(ctx: Context, bsr_vals, x, y=None, stream=None):
    y = torch.empty_like(x) if y is None else y
    _check(_lib.vms_bsr_spmv(ctx.handle, _ptr(bsr_vals), _ptr(x), _ptr(y), _stream(stream)), ctx.handle)
    return y


def vms_gmres_solve(ctx: Context, bsr_vals, b, x, opts: SolveOpts, stream=None, allow_noconv=False):
    info = SolveInfo()
    rc = _lib.vms_gmres_solve(ctx.handle, _ptr(bsr_vals), _ptr(b), _ptr(x), ctypes.byref(opts),
                              ctypes.byref(info), _stream(stream))
    _check(rc, ctx.handle, allow=(VMS_ENOCONV_GMRES,) if allow_noconv else ())
    return rc, info


def vms_newton_step(ctx: Context, u, beta, Re, dt=0.0, u_prev=None, body=None, lin: SolveOpts = None,
                    stream=None):
    opts = NewtonOpts(lin if lin is not None else solve_opts())
    info = NewtonInfo()
    rc = _lib.vms_newton_step(ctx.handle, _ptr(u), _ptr(beta), _ptr(u_prev), float(Re), float(dt), _ptr(body),
                              ctypes.byref(opts), ctypes.byref(info), _stream(stream))
    _check(rc, ctx.handle)
    return info


def vms_set_linearization(ctx: Context, kind):
    """kind: VMS_LIN_NEWTON (consistent tangent) or VMS_LIN_PICARD (advecting velocity held)."""
    _check(_lib.vms_set_linearization(ctx.handle, int(kind)), ctx.handle)


def vms_full_assemble(ctx: Context, u, beta, Re, dt=0.0, u_prev=None, body=None, bsr_vals=None, rhs=None,
                      rnorm=None, stream=None):
    bsr_vals = ctx.new_full_bsr() if bsr_vals is None else bsr_vals
    rhs = ctx.new_full_vec() if rhs is None else rhs
    rnorm = torch.zeros(1, dtype=torch.float64, device=ctx.device) if rnorm is None else rnorm
    _check(_lib.vms_full_assemble(ctx.handle, _ptr(u), _ptr(u_prev), _ptr(beta), float(Re), float(dt),
                                  _ptr(body), _ptr(bsr_vals), _ptr(rhs), _ptr(rnorm), _stream(stream)),
           ctx.handle)
    return bsr_vals, rhs, rnorm


def vms_full_newton_step(ctx: Context, u, beta, Re, dt=0.0, u_prev=None, body=None, lin: SolveOpts = None,
                         stream=None):
    opts = NewtonOpts(lin if lin is not None else solve_opts())
    info = NewtonInfo()
    rc = _lib.vms_full_newton_step(ctx.handle, _ptr(u), _ptr(beta), _ptr(u_prev), float(Re), float(dt),
                                   _ptr(body), ctypes.byref(opts), ctypes.byref(info), _stream(stream))
    _check(rc, ctx.handle)
    return info


def vms_pc_features(ctx: Context, bsr_vals, feats=None, stream=None):
    feats = torch.empty((ctx.n_nodes, PC_NIN), dtype=torch.float32, device=ctx.device) if feats is None else feats
    _check(_lib.vms_pc_features(ctx.handle, _ptr(bsr_vals), _ptr(feats), _stream(stream)), ctx.handle)
    return feats


def vms_pc_blocks(ctx: Context, bsr_vals, weights=None, P=None, stream=None):
    P = torch.empty((ctx.n_nodes, 16), dtype=torch.float32, device=ctx.device) if P is None else P
    _check(_lib.vms_pc_blocks(ctx.handle, _ptr(bsr_vals), _ptr(weights), _ptr(P), _stream(stream)), ctx.handle)
    return P


def vms_pc_train_step(ctx: Context, bsr_vals, r_batch, weights, adam_state, step, lr, grad_out=None,
                      loss_out=None, stream=None):
    nbatch = int(r_batch.shape[0])
    _check(_lib.vms_pc_train_step(ctx.handle, _ptr(bsr_vals), _ptr(r_batch), nbatch, _ptr(weights),
                                  _ptr(adam_state), int(step), float(lr), _ptr(grad_out), _ptr(loss_out),
                                  _stream(stream)), ctx.handle)


def vms_profile(ctx: Context, enable=True, phases=None, every=1):
    """Times the launches of the named phases (all phases when None), every `every`-th
    launch of each; enable=False stops."""
    if not enable:
        mask = 0
    elif phases is None:
        mask = (1 << len(PHASES)) - 1
    else:
        mask = 0
        for p in ([phases] if isinstance(phases, str) else phases):
            mask |= 1 << PHASES.index(p)
    _check(_lib.vms_profile(ctx.handle, mask, int(every)), ctx.handle)


def vms_profile_read(ctx: Context):
    """{phase: (ms, launches, algorithmic bytes)} accumulated since vms_profile."""
    n = len(PHASES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    byt = (ctypes.c_double * n)()
    _check(_lib.vms_profile_read(ctx.handle, ms, cnt, byt), ctx.handle)
    return {PHASES[i]: (ms[i], int(cnt[i]), byt[i]) for i in range(n)}
