"""Python binding of libhf, the MI355X (gfx950) Newton step of the
fully-coupled DG/CZM + lubrication hydraulic-fracture method.

Argument marshalling only: every step of the Newton iteration runs in the
library's HIP kernels.  Importing the package never falls back to a CPU
path: ``load()`` raises if libhf.so is missing, and ``Context`` raises if no
GPU is visible.  Device buffers may be passed as torch tensors (their
``data_ptr()``) to the ``*_device`` calls; torch is not needed otherwise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhf.so")

HF_OK, HF_EINVAL, HF_ENOMEM, HF_EDEVICE, HF_ESTATE, HF_ESINGULAR, HF_ENOCONV, HF_ENONFINITE = \
    0, -1, -2, -3, -4, -5, -6, -7
HF_FP64, HF_FP32_IR = 0, 1
STATUS_NAMES = {0: "HF_OK", -1: "HF_EINVAL", -2: "HF_ENOMEM", -3: "HF_EDEVICE", -4: "HF_ESTATE",
                -5: "HF_ESINGULAR", -6: "HF_ENOCONV", -7: "HF_ENONFINITE"}

# every symbol include/hf.h declares
EXPORTS = [
    "hf_default_options", "hf_create", "hf_destroy", "hf_last_error", "hf_set_options",
    "hf_instance_count",
    "hf_upload_mesh", "hf_get_faces", "hf_upload_interfaces", "hf_set_material",
    "hf_set_injection", "hf_finalize", "hf_get_sizes", "hf_get_pnodes", "hf_set_state",
    "hf_get_state", "hf_set_state_device", "hf_get_state_device", "hf_assemble", "hf_solve",
    "hf_newton_step", "hf_newton_solve", "hf_staggered_step", "hf_end_load_step",
    "hf_get_interface_traction", "hf_detect_activation", "hf_set_history", "hf_get_history",
    "hf_initial_guess", "hf_get_residual",
    "hf_get_block_rows", "hf_get_coupling", "hf_get_increment", "hf_apply_jacobian",
    "hf_get_profile", "hf_reset_profile", "hf_get_tuning", "hf_set_tuning", "hf_autotune",
    "hf_get_block_inverse", "hf_apply_preconditioned", "hf_apply_preconditioned_noalloc",
]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("gmres_m", C.c_int), ("gmres_maxit", C.c_int),
                ("ir_maxit", C.c_int), ("newton_maxit", C.c_int), ("rtol", C.c_double),
                ("rtol_inner", C.c_double), ("newton_tol", C.c_double), ("b_stab", C.c_double),
                ("p_cutoff", C.c_double), ("cutoff_on", C.c_int), ("device", C.c_int),
                ("profile", C.c_int), ("use_graphs", C.c_int), ("mfma_inverse", C.c_int),
                ("ir_inner_cycles", C.c_int), ("ir_stall_steps", C.c_int),
                ("incremental_assembly", C.c_int),
                ("fold_preconditioner", C.c_int), ("two_level", C.c_int), ("coarse_leaf", C.c_int),
                ("coarse_reuse", C.c_int), ("coarse_fp32", C.c_int),
                ("scale_fluid_rows", C.c_int), ("cohesive_unloading", C.c_int),
                ("stream", C.c_void_p)]


class Material(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("sigma_c", C.c_double),
                ("G_c", C.c_double), ("mu", C.c_double), ("dt", C.c_double)]


class Sizes(C.Structure):
    _fields_ = [("n_elem", C.c_int64), ("nodes_per_elem", C.c_int64), ("n_u", C.c_int64),
                ("n_p", C.c_int64), ("n_face", C.c_int64), ("n_blocks", C.c_int64),
                ("u_offset", C.c_int64), ("p_offset", C.c_int64), ("n_total", C.c_int64),
                ("dim", C.c_int32), ("order", C.c_int32), ("nq_face", C.c_int32),
                ("block_size", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("gmres_iters", C.c_int), ("ir_steps", C.c_int), ("restarts", C.c_int),
                ("status", C.c_int), ("fp64_iters", C.c_int), ("true_relres", C.c_double),
                ("seconds", C.c_double), ("relres_u", C.c_double), ("relres_p", C.c_double)]


class NewtonStats(C.Structure):
    _fields_ = [("lin", SolveStats), ("du_rel", C.c_double), ("dp_rel", C.c_double),
                ("res_norm", C.c_double), ("iterations", C.c_int), ("converged", C.c_int),
                ("status", C.c_int), ("reserved", C.c_int)]


class Tuning(C.Structure):
    _fields_ = [("spmv_var", C.c_int), ("prec_var", C.c_int), ("ortho_var", C.c_int),
                ("reorth", C.c_int), ("gmres_m", C.c_int), ("dense_wide_min", C.c_int),
                ("inv_var", C.c_int), ("reserved", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k in ("spmv_var", "prec_var", "ortho_var", "reorth",
                                               "gmres_m", "inv_var")}


class Profile(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("ms_assemble", "ms_blockinv", "ms_spmv64", "ms_spmv32",
                                           "ms_precond", "ms_ortho")] + \
               [(n, C.c_int64) for n in ("n_assemble", "n_blockinv", "n_spmv64", "n_spmv32",
                                          "n_precond", "n_ortho", "n_inv_mfma",
                                          "n_inv_fallback")] + \
               [("ms_resid", C.c_double), ("n_resid", C.c_int64), ("n_unfold", C.c_int64),
                ("n_mgrow", C.c_int64), ("n_ir_rise", C.c_int64), ("n_tl_builds", C.c_int64),
                ("n_tl_fail", C.c_int64), ("n_tl_factor", C.c_int64)]


class HFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libhf.so (built by ``paper_1911_10275_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not built: run python -m paper_1911_10275_amd.build")
    # torch ships its own HIP runtime under the same soname as ROCm's; loading
    # torch first makes libhf bind to that one copy instead of a second runtime
    # that torch could not initialise alongside.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    P = C.POINTER
    vp = C.c_void_p
    sig = {
        "hf_default_options": (None, [P(Options)]),
        "hf_create": (C.c_int, [P(Options), P(vp)]),
        "hf_destroy": (None, [vp]),
        "hf_last_error": (C.c_char_p, [vp]),
        "hf_set_options": (C.c_int, [vp, P(Options)]),
        "hf_instance_count": (C.c_int, [vp, P(C.c_int32)]),
        "hf_upload_mesh": (C.c_int, [vp, C.c_int, C.c_int, C.c_int64, vp, C.c_int64, vp, vp,
                                     P(C.c_int32)]),
        "hf_get_faces": (C.c_int, [vp, C.c_int32, P(C.c_int64), vp, vp, P(C.c_int32)]),
        "hf_upload_interfaces": (C.c_int, [vp, C.c_int32, vp, vp]),
        "hf_set_material": (C.c_int, [vp, C.c_int32, P(Material)]),
        "hf_set_injection": (C.c_int, [vp, C.c_int32, C.c_int32, vp, vp]),
        "hf_finalize": (C.c_int, [vp]),
        "hf_get_sizes": (C.c_int, [vp, C.c_int32, P(Sizes)]),
        "hf_get_pnodes": (C.c_int, [vp, C.c_int32, vp]),
        "hf_set_state": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
        "hf_get_state": (C.c_int, [vp, C.c_int32, vp, vp, vp, vp]),
        "hf_set_state_device": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
        "hf_get_state_device": (C.c_int, [vp, C.c_int32, vp, vp]),
        "hf_assemble": (C.c_int, [vp, P(C.c_double)]),
        "hf_solve": (C.c_int, [vp, P(SolveStats)]),
        "hf_newton_step": (C.c_int, [vp, P(NewtonStats)]),
        "hf_newton_solve": (C.c_int, [vp, P(NewtonStats)]),
        "hf_staggered_step": (C.c_int, [vp, P(C.c_int32), P(C.c_double), P(NewtonStats)]),
        "hf_get_interface_traction": (C.c_int, [vp, C.c_int32, P(C.c_double)]),
        "hf_detect_activation": (C.c_int, [vp, C.c_int32, P(C.c_uint8), P(C.c_uint8), P(C.c_int64)]),
        "hf_end_load_step": (C.c_int, [vp]),
        "hf_set_history": (C.c_int, [vp, C.c_int32, vp]),
        "hf_get_history": (C.c_int, [vp, C.c_int32, vp]),
        "hf_initial_guess": (C.c_int, [vp, P(C.c_double)]),
        "hf_get_residual": (C.c_int, [vp, C.c_int32, vp, vp]),
        "hf_get_block_rows": (C.c_int, [vp, C.c_int32, C.c_int64, vp, vp, vp]),
        "hf_get_coupling": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
        "hf_get_increment": (C.c_int, [vp, C.c_int32, vp, vp]),
        "hf_apply_jacobian": (C.c_int, [vp, C.c_int, vp, vp]),
        "hf_apply_preconditioned": (C.c_int, [vp, C.c_int, C.c_int, vp, vp]),
        "hf_apply_preconditioned_noalloc": (C.c_int, [vp, C.c_int, vp, vp]),
        "hf_get_profile": (C.c_int, [vp, P(Profile)]),
        "hf_reset_profile": (C.c_int, [vp]),
        "hf_get_tuning": (C.c_int, [vp, P(Tuning)]),
        "hf_get_block_inverse": (C.c_int, [vp, C.c_int32, C.c_int64, vp, C.c_int, vp]),
        "hf_set_tuning": (C.c_int, [vp, P(Tuning)]),
        "hf_autotune": (C.c_int, [vp, C.c_int, C.c_char_p, P(Tuning)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def default_options(**kw) -> Options:
    lib = load()
    o = Options()
    lib.hf_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Context:
    """One or more fracture instances on one GPU (owns the library context).

    Per-instance calls take ``inst`` (default 0).  The compute calls work on
    every instance at once; with one instance they return scalars / single
    stats, with several a numpy array / list (one entry per instance).  With
    ``check=False`` they return the per-instance results even when some
    instance failed (inspect ``.status``)."""

    def __init__(self, **options):
        self.lib = load()
        self.opt = default_options(**options)
        h = C.c_void_p()
        st = self.lib.hf_create(C.byref(self.opt), C.byref(h))
        if st != HF_OK:
            raise HFError(st, "hf_create failed (is a gfx950 GPU visible?)")
        self.h = h
        self.sizes = None      # of instance 0, after finalize
        self.isizes = []       # of every instance, after finalize

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.hf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st, what):
        if st != HF_OK:
            raise HFError(st, f"{what}: {self.lib.hf_last_error(self.h).decode()}")

    def set_options(self, **kw):
        for k, v in kw.items():
            setattr(self.opt, k, v)
        self._check(self.lib.hf_set_options(self.h, C.byref(self.opt)), "hf_set_options")

    @property
    def n_inst(self) -> int:
        n = C.c_int32()
        self._check(self.lib.hf_instance_count(self.h, C.byref(n)), "hf_instance_count")
        return n.value

    # -- setup ---------------------------------------------------------------
    def upload_mesh(self, dim, order, xyz, elem, dirichlet_vert=None) -> int:
        xyz = _arr(xyz, np.float64)
        elem = _arr(elem, np.int32)
        dv = None if dirichlet_vert is None else _arr(dirichlet_vert, np.uint8)
        inst = C.c_int32()
        self._check(self.lib.hf_upload_mesh(self.h, dim, order, xyz.shape[0], _ptr(xyz),
                                            elem.shape[0], _ptr(elem), _ptr(dv), C.byref(inst)),
                    "hf_upload_mesh")
        return inst.value

    def faces(self, inst=0):
        nf = C.c_int64()
        nq = C.c_int32()
        self._check(self.lib.hf_get_faces(self.h, inst, C.byref(nf), None, None, C.byref(nq)),
                    "hf_get_faces")
        s = self.get_sizes(inst)
        fv = np.empty((nf.value, s.dim), dtype=np.int32)
        fe = np.empty((nf.value, 2), dtype=np.int32)
        self._check(self.lib.hf_get_faces(self.h, inst, C.byref(nf), _ptr(fv), _ptr(fe), None),
                    "hf_get_faces")
        return fv, fe, nq.value

    def upload_interfaces(self, qp_state=None, beta=None, inst=0):
        q = None if qp_state is None else _arr(qp_state, np.uint8)
        b = None if beta is None else _arr(beta, np.uint8)
        self._check(self.lib.hf_upload_interfaces(self.h, inst, _ptr(q), _ptr(b)),
                    "hf_upload_interfaces")

    def set_material(self, E, nu, sigma_c, G_c, mu, dt, inst=0):
        m = Material(E, nu, sigma_c, G_c, mu, dt)
        self._check(self.lib.hf_set_material(self.h, inst, C.byref(m)), "hf_set_material")

    def set_injection(self, vert, q0, inst=0):
        v = _arr(vert, np.int64)
        q = _arr(q0, np.float64)
        self._check(self.lib.hf_set_injection(self.h, inst, len(v), _ptr(v), _ptr(q)),
                    "hf_set_injection")

    def finalize(self):
        self._check(self.lib.hf_finalize(self.h), "hf_finalize")
        self.isizes = [self.get_sizes(b) for b in range(self.n_inst)]
        self.sizes = self.isizes[0]

    def get_sizes(self, inst=0) -> Sizes:
        s = Sizes()
        self._check(self.lib.hf_get_sizes(self.h, inst, C.byref(s)), "hf_get_sizes")
        return s

    def pnodes(self, inst=0):
        s = self.get_sizes(inst)
        k = np.empty((s.n_p, 2), dtype=np.int64)
        self._check(self.lib.hf_get_pnodes(self.h, inst, _ptr(k)), "hf_get_pnodes")
        return k

    # -- state ---------------------------------------------------------------
    def set_state(self, u, p, w_old=None, inst=0):
        u = _arr(u, np.float64)
        p = _arr(p, np.float64)
        w = None if w_old is None else _arr(w_old, np.float64)
        self._check(self.lib.hf_set_state(self.h, inst, _ptr(u), _ptr(p), _ptr(w)),
                    "hf_set_state")

    def get_state(self, inst=0):
        s = self.isizes[inst]
        u = np.empty(s.n_u)
        p = np.empty(s.n_p)
        w = np.empty((s.n_face, s.nq_face))
        wo = np.empty((s.n_face, s.nq_face))
        self._check(self.lib.hf_get_state(self.h, inst, _ptr(u), _ptr(p), _ptr(w), _ptr(wo)),
                    "hf_get_state")
        return u, p, w, wo

    def set_history(self, w_max, inst=0):
        """Unloading history w_max per face point (cohesive_unloading)."""
        w = _arr(w_max, np.float64)
        self._check(self.lib.hf_set_history(self.h, inst, _ptr(w)), "hf_set_history")

    def get_history(self, inst=0):
        s = self.isizes[inst]
        w = np.empty((s.n_face, s.nq_face))
        self._check(self.lib.hf_get_history(self.h, inst, _ptr(w)), "hf_get_history")
        return w

    def set_state_device(self, u_ptr, p_ptr, w_old_ptr=None, inst=0):
        self._check(self.lib.hf_set_state_device(self.h, inst, C.c_void_p(u_ptr),
                                                 C.c_void_p(p_ptr),
                                                 None if w_old_ptr is None else C.c_void_p(w_old_ptr)),
                    "hf_set_state_device")

    # -- the Newton step (all instances) -------------------------------------------
    def _one(self, arr):
        return arr[0] if len(arr) == 1 else arr

    def assemble(self):
        r = np.zeros(self.n_inst)
        self._check(self.lib.hf_assemble(self.h, r.ctypes.data_as(C.POINTER(C.c_double))),
                    "hf_assemble")
        return float(r[0]) if len(r) == 1 else r

    def solve(self, check=True):
        st = (SolveStats * self.n_inst)()
        rc = self.lib.hf_solve(self.h, st)
        if check:
            self._check(rc, "hf_solve")
        return self._one(list(st))

    def newton_step(self, check=True):
        st = (NewtonStats * self.n_inst)()
        rc = self.lib.hf_newton_step(self.h, st)
        if check:
            self._check(rc, "hf_newton_step")
        return self._one(list(st))

    def newton_solve(self, check=True):
        st = (NewtonStats * self.n_inst)()
        rc = self.lib.hf_newton_solve(self.h, st)
        if check:
            self._check(rc, "hf_newton_solve")
        return self._one(list(st))

    def staggered_step(self, dir_node, dir_value=None, check=True):
        """One iteration of the staggered comparison scheme; dir_node /
        dir_value: the essential pressure condition of each instance
        (instance-local pressure-node index and value; scalars for one
        instance)."""
        node = np.ascontiguousarray(np.atleast_1d(dir_node), dtype=np.int32)
        val = None if dir_value is None else np.ascontiguousarray(np.atleast_1d(dir_value), dtype=np.float64)
        if len(node) != self.n_inst or (val is not None and len(val) != self.n_inst):
            raise ValueError("one dir_node (and dir_value) per instance")
        st = (NewtonStats * self.n_inst)()
        rc = self.lib.hf_staggered_step(self.h, node.ctypes.data_as(C.POINTER(C.c_int32)),
                                        None if val is None else val.ctypes.data_as(C.POINTER(C.c_double)),
                                        st)
        if check:
            self._check(rc, "hf_staggered_step")
        return self._one(list(st))

    def end_load_step(self):
        self._check(self.lib.hf_end_load_step(self.h), "hf_end_load_step")

    def interface_traction(self, inst=0):
        """DG normal traction at every face point, (n_face, nq_face)."""
        s = self.isizes[inst]
        tn = np.empty((s.n_face, s.nq_face))
        self._check(self.lib.hf_get_interface_traction(self.h, inst, tn.ctypes.data_as(C.POINTER(C.c_double))),
                    "hf_get_interface_traction")
        return tn

    def detect_activation(self, inst=0):
        """New interface states after the activation checks: (qp_state, beta,
        points newly activated, faces newly fluid)."""
        s = self.isizes[inst]
        qp = np.empty((s.n_face, s.nq_face), dtype=np.uint8)
        beta = np.empty(s.n_face, dtype=np.uint8)
        n = np.zeros(2, dtype=np.int64)
        self._check(self.lib.hf_detect_activation(self.h, inst, qp.ctypes.data_as(C.POINTER(C.c_uint8)),
                                                  beta.ctypes.data_as(C.POINTER(C.c_uint8)),
                                                  n.ctypes.data_as(C.POINTER(C.c_int64))),
                    "hf_detect_activation")
        return qp, beta, int(n[0]), int(n[1])

    def initial_guess(self):
        """Uniform-pressure elastic predictor for the first load step; returns p0
        (an array with one entry per instance when there are several)."""
        p0 = np.zeros(self.n_inst)
        self._check(self.lib.hf_initial_guess(self.h, p0.ctypes.data_as(C.POINTER(C.c_double))),
                    "hf_initial_guess")
        return float(p0[0]) if len(p0) == 1 else p0

    # -- inspection ------------------------------------------------------------------
    def residual(self, inst=0):
        s = self.isizes[inst]
        ru = np.empty(s.n_u)
        rp = np.empty(s.n_p)
        self._check(self.lib.hf_get_residual(self.h, inst, _ptr(ru), _ptr(rp)), "hf_get_residual")
        return ru, rp

    def block_rows(self, elems, inst=0):
        s = self.isizes[inst]
        e = _arr(elems, np.int32)
        ns = s.dim + 2
        cols = np.empty((len(e), ns), dtype=np.int32)
        blocks = np.empty((len(e), ns, s.block_size, s.block_size))
        self._check(self.lib.hf_get_block_rows(self.h, inst, len(e), _ptr(e), _ptr(cols),
                                               _ptr(blocks)), "hf_get_block_rows")
        return cols, blocks

    def coupling(self, inst=0):
        s = self.isizes[inst]
        B = np.empty((s.n_u, s.n_p))
        Cm = np.empty((s.n_p, s.n_u))
        D = np.empty((s.n_p, s.n_p))
        self._check(self.lib.hf_get_coupling(self.h, inst, _ptr(B), _ptr(Cm), _ptr(D)),
                    "hf_get_coupling")
        return B, Cm, D

    def block_inverse(self, elems, precision=HF_FP64, inst=0):
        """Preconditioner inverses of the given element blocks (row-major)."""
        s = self.isizes[inst]
        e = _arr(elems, np.int32)
        out = np.empty((len(e), s.block_size, s.block_size))
        self._check(self.lib.hf_get_block_inverse(self.h, inst, len(e), _ptr(e), precision,
                                                  _ptr(out)), "hf_get_block_inverse")
        return out

    def increment(self, inst=0):
        s = self.isizes[inst]
        du = np.empty(s.n_u)
        dp = np.empty(s.n_p)
        self._check(self.lib.hf_get_increment(self.h, inst, _ptr(du), _ptr(dp)),
                    "hf_get_increment")
        return du, dp

    def apply_jacobian(self, x_ptr, y_ptr, precision=HF_FP64):
        self._check(self.lib.hf_apply_jacobian(self.h, precision, C.c_void_p(x_ptr),
                                               C.c_void_p(y_ptr)), "hf_apply_jacobian")

    def apply_preconditioned(self, x_ptr, y_ptr, precision=HF_FP64, folded=1):
        self._check(self.lib.hf_apply_preconditioned(self.h, precision, int(folded), C.c_void_p(x_ptr),
                                                     C.c_void_p(y_ptr)), "hf_apply_preconditioned")

    def apply_preconditioned_noalloc(self, x_ptr, y_ptr, precision=HF_FP64):
        """The folded y = J M^-1 x with the library's fixed scratch array
        (no allocation, no synchronisation)."""
        self._check(self.lib.hf_apply_preconditioned_noalloc(self.h, precision, C.c_void_p(x_ptr),
                                                             C.c_void_p(y_ptr)),
                    "hf_apply_preconditioned_noalloc")

    def profile(self) -> Profile:
        p = Profile()
        self._check(self.lib.hf_get_profile(self.h, C.byref(p)), "hf_get_profile")
        return p

    def reset_profile(self):
        self._check(self.lib.hf_reset_profile(self.h), "hf_reset_profile")

    # -- tuning --------------------------------------------------------------------------
    def tuning(self) -> Tuning:
        t = Tuning()
        self._check(self.lib.hf_get_tuning(self.h, C.byref(t)), "hf_get_tuning")
        return t

    def set_tuning(self, **kw):
        t = self.tuning()
        for k, v in kw.items():
            if k not in Tuning().as_dict() and k != "dense_wide_min":
                raise KeyError(k)
            setattr(t, k, v)
        self._check(self.lib.hf_set_tuning(self.h, C.byref(t)), "hf_set_tuning")
        self.opt.gmres_m = t.gmres_m

    def autotune(self, level=0, cache_path=None) -> Tuning:
        """Pick kernel schedules (level 0) and restart length / orthogonalisation
        (level 1) by timing them on the assembled system, or apply the cached
        choice without timing (level -1); see hf_autotune."""
        t = Tuning()
        cp = None if cache_path is None else os.fsencode(cache_path)
        self._check(self.lib.hf_autotune(self.h, level, cp, C.byref(t)), "hf_autotune")
        self.opt.gmres_m = t.gmres_m
        return t


def _upload_problem(ctx: Context, prob) -> int:
    inst = ctx.upload_mesh(prob.dim, prob.order, prob.xyz, prob.elem, prob.dirichlet_vert)
    fv, _, nq = ctx.faces(inst)
    index = {tuple(r): i for i, r in enumerate(fv.tolist())}
    qs = np.zeros((len(fv), nq), dtype=np.uint8)
    beta = np.zeros(len(fv), dtype=np.uint8)
    for key, st, bt in zip(np.asarray(prob.crack_faces), np.asarray(prob.crack_state),
                           np.asarray(prob.crack_beta)):
        f = index[tuple(sorted(int(v) for v in key))]
        qs[f, :] = st
        beta[f] = bt
    ctx.upload_interfaces(qs, beta, inst=inst)
    m = prob.material
    ctx.set_material(m.E, m.nu, m.sigma_c, m.G_c, m.mu, m.dt, inst=inst)
    ctx.set_injection(np.asarray(prob.src_vert), np.asarray(prob.src_q0), inst=inst)
    return inst


def context_for_problems(probs, b_stab: float = 10.0, **options) -> Context:
    """Build a finalized Context holding one instance per problem.  A problem
    has attributes dim, order, xyz, elem, dirichlet_vert, crack_faces (vertex
    ids), crack_state, crack_beta, src_vert, src_q0 and material (E, nu,
    sigma_c, G_c, mu, dt).  Crack faces are located among the library's
    interior faces by their vertex ids; every integration point of a crack
    face gets its state."""
    ctx = Context(b_stab=b_stab, **options)
    for prob in probs:
        _upload_problem(ctx, prob)
    ctx.finalize()
    return ctx


def context_for_problem(prob, b_stab: float = 10.0, **options) -> Context:
    """A finalized single-instance Context (see ``context_for_problems``)."""
    return context_for_problems([prob], b_stab=b_stab, **options)
