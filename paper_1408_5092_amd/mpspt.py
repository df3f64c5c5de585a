"""Python binding of libmpspt.so (the HIP MPS-PT library).

Argument marshalling only: every step of the sweep runs in the library's
gfx950 kernels.  The names mirror include/mpspt.h.  The stream handed to the
library is PyTorch's current HIP stream when torch is importable.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpspt.so")
# launch-shape choice recorded by python -m paper_1408_5092_amd.autotune
TUNING_PATH = os.path.join(_HERE, "tuning.json")

STATUS = {0: "MPSPT_OK", -1: "MPSPT_E_ARG", -2: "MPSPT_E_QN", -3: "MPSPT_E_NOMEM", -4: "MPSPT_E_HIP",
          -5: "MPSPT_E_INDEFINITE", -6: "MPSPT_E_STATE", -7: "MPSPT_E_NODEV"}

EXPORTED = ["mpspt_create", "mpspt_destroy", "mpspt_last_error", "mpspt_load_integrals",
            "mpspt_load_integrals_eri", "mpspt_load_h0_partition", "mpspt_load_psi0",
            "mpspt_restrict_virtual", "mpspt_load_psi1_guess", "mpspt_ground_state", "mpspt_sweep", "mpspt_profile", "mpspt_set_tuning", "mpspt_get_tuning",
            "mpspt_kernel_stats", "mpspt_get_trace", "mpspt_get_bond",
            "mpspt_get_site", "mpspt_mpo_dense", "mpspt_mpo_dims", "mpspt_precond_set", "mpspt_precond_get",
            "mpspt_mlp_grad", "mpspt_mlp_train_step", "mpspt_harvest", "mpspt_harvest_get"]
MLP_PARAMS, MLP_INPUTS = 4801, 8


class MPSPTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class SweepParams(C.Structure):
    _fields_ = [("M1", C.c_int32), ("n_sweeps", C.c_int32), ("max_sweeps", C.c_int32),
                ("e_tol", C.c_double), ("cg_rel_tol", C.c_double), ("cg_max_iter", C.c_int32),
                ("compute_e3", C.c_int32), ("precond", C.c_int32), ("precision", C.c_int32),
                ("inner_rel_tol", C.c_double)]


class Result(C.Structure):
    _fields_ = [("e0", C.c_double), ("e2", C.c_double), ("e3", C.c_double),
                ("n_sweeps_done", C.c_int32), ("n_steps", C.c_int32),
                ("e2_sweep", C.c_double * 64), ("max_discarded", C.c_double),
                ("cg_iters", C.c_int64), ("sigma_calls", C.c_int64),
                ("sigma_flops", C.c_double), ("sigma_bytes", C.c_double),
                ("t_total_s", C.c_double), ("flags", C.c_int32), ("t_phase", C.c_double * 6),
                ("plan_builds", C.c_int64), ("plan_hits", C.c_int64),
                ("sigma_lo_calls", C.c_int64), ("refinements", C.c_int64)]


_lib = None


def load_library(path: str | None = None):
    """Load the built library (raises if it has not been built)."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or LIB_PATH
    # PyTorch ships its own HIP runtime; loading it first makes the library
    # bind to that same runtime instead of starting a second one
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build the HIP library first (python __graft_entry__.py build)")
    lib = C.CDLL(p)
    P, I, D = C.c_void_p, C.c_int32, C.c_double
    dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)
    lib.mpspt_create.argtypes = [C.c_int, P, C.POINTER(P)]
    lib.mpspt_destroy.argtypes = [P]
    lib.mpspt_destroy.restype = None
    lib.mpspt_last_error.argtypes = [P]
    lib.mpspt_last_error.restype = C.c_char_p
    lib.mpspt_load_integrals.argtypes = [P, I, I, dp, I, dp]
    lib.mpspt_load_integrals_eri.argtypes = [P, I, I, dp, dp]
    lib.mpspt_load_h0_partition.argtypes = [P, I, dp]
    lib.mpspt_load_psi0.argtypes = [P, I, I, ip, ip, C.POINTER(dp)]
    lib.mpspt_load_psi1_guess.argtypes = [P, ip, ip, C.POINTER(dp)]
    lib.mpspt_ground_state.argtypes = [P, I, I, ip, ip, C.POINTER(dp), I, I, D, dp]
    lib.mpspt_profile.argtypes = [P, I]
    lib.mpspt_kernel_stats.argtypes = [P, I, dp, C.POINTER(C.c_int64), dp, dp]
    lib.mpspt_sweep.argtypes = [P, C.POINTER(SweepParams), C.POINTER(Result)]
    lib.mpspt_get_trace.argtypes = [P, I, dp, ip, dp, dp, ip]
    lib.mpspt_get_bond.argtypes = [P, I, I, I, ip, ip]
    lib.mpspt_get_site.argtypes = [P, I, I, C.c_size_t, dp, ip]
    lib.mpspt_mpo_dense.argtypes = [I, I, dp, dp, dp, I, dp, C.c_size_t]
    lib.mpspt_mpo_dims.argtypes = [I, I, dp, dp, dp, I, ip, I]
    fp = C.POINTER(C.c_float)
    lib.mpspt_precond_set.argtypes = [P, fp, I]
    lib.mpspt_precond_get.argtypes = [P, fp, I]
    lib.mpspt_mlp_grad.argtypes = [P, fp, fp, I, fp, fp]
    lib.mpspt_mlp_train_step.argtypes = [P, fp, fp, I, C.c_float, fp]
    lib.mpspt_harvest.argtypes = [P, I]
    lib.mpspt_harvest_get.argtypes = [P, C.c_int64, fp, fp, C.POINTER(C.c_int64)]
    for name in EXPORTED:
        if name not in ("mpspt_destroy", "mpspt_last_error"):
            getattr(lib, name).restype = C.c_int
    if path is None:
        _lib = lib
    return lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _mps_args(bonds, sites):
    dims = np.array([sum(d for _, d in b) for b in bonds], dtype=np.int32)
    lab = []
    for b in bonds:
        for (n, s), d in b:
            lab += [n, s] * d
    qn = np.array(lab, dtype=np.int32)
    keep = [np.ascontiguousarray(s, dtype=np.float64) for s in sites]
    ptrs = (C.POINTER(C.c_double) * len(keep))(*[k.ctypes.data_as(C.POINTER(C.c_double)) for k in keep])
    return dims, qn, keep, ptrs


def current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return C.c_void_p(None)


class Context:
    """One library context on one HIP device."""

    def __init__(self, device: int = 0, stream=None, lib=None):
        self.lib = lib or load_library()
        h = C.c_void_p()
        st = self.lib.mpspt_create(device, stream if stream is not None else current_stream(), C.byref(h))
        if st != 0:
            raise MPSPTError(st, self.lib.mpspt_last_error(None).decode())
        self.h = h
        if os.path.exists(TUNING_PATH):
            with open(TUNING_PATH) as f:
                t = json.load(f)["choice"]
            self.set_tuning(t["wide_chunks"], t["kseg_min"], t["kseg_div"], t.get("split_waves", 4))

    def close(self):
        if getattr(self, "h", None):
            self.lib.mpspt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ok(self, st):
        if st != 0:
            raise MPSPTError(st, self.lib.mpspt_last_error(self.h).decode())

    # ---- mirrors of the C entry points
    def load_integrals(self, k_a, k_v, h, B):
        h, hp = _d(h)
        B, Bp = _d(B)
        self._ok(self.lib.mpspt_load_integrals(self.h, k_a, k_v, hp, B.shape[0], Bp))

    def load_integrals_eri(self, k_a, k_v, h, eri):
        h, hp = _d(h)
        e, ep = _d(eri)
        self._ok(self.lib.mpspt_load_integrals_eri(self.h, k_a, k_v, hp, ep))

    def load_h0_partition(self, eps_virt, kind=0):
        e, ep = _d(eps_virt)
        self._ok(self.lib.mpspt_load_h0_partition(self.h, kind, ep))

    def load_psi0(self, n_elec, two_sz, bonds, sites):
        dims, qn, keep, ptrs = _mps_args(bonds, sites)
        self._ok(self.lib.mpspt_load_psi0(self.h, n_elec, two_sz, dims.ctypes.data_as(C.POINTER(C.c_int32)),
                                          qn.ctypes.data_as(C.POINTER(C.c_int32)), ptrs))

    def ground_state(self, n_elec, two_sz, bonds, sites, M0, n_sweeps=0, e_tol=1e-10):
        dims, qn, keep, ptrs = _mps_args(bonds, sites)
        e = C.c_double()
        self._ok(self.lib.mpspt_ground_state(self.h, n_elec, two_sz, dims.ctypes.data_as(C.POINTER(C.c_int32)),
                                             qn.ctypes.data_as(C.POINTER(C.c_int32)), ptrs, M0, n_sweeps, e_tol,
                                             C.byref(e)))
        return e.value

    def restrict_virtual(self, masks=None):
        """Per virtual site, a bit mask of the electron counts it may hold
        (None: no restriction); see mpspt_restrict_virtual."""
        if masks is None:
            self._ok(self.lib.mpspt_restrict_virtual(self.h, None))
            return
        m = np.ascontiguousarray(masks, dtype=np.int32)
        self._ok(self.lib.mpspt_restrict_virtual(self.h, m.ctypes.data_as(C.POINTER(C.c_int32))))

    def load_psi1_guess(self, bonds, sites):
        dims, qn, keep, ptrs = _mps_args(bonds, sites)
        self._ok(self.lib.mpspt_load_psi1_guess(self.h, dims.ctypes.data_as(C.POINTER(C.c_int32)),
                                                qn.ctypes.data_as(C.POINTER(C.c_int32)), ptrs))

    def sweep(self, M1, n_sweeps=0, max_sweeps=10, e_tol=1e-9, cg_rel_tol=1e-10, cg_max_iter=500,
              compute_e3=True, precond=0, precision=0, inner_rel_tol=0.0):
        """precision: 0 FP64, 1 FP32, 2 BF16x3 sigma inside CG (FP64 refinement)."""
        p = SweepParams(M1, n_sweeps, max_sweeps, e_tol, cg_rel_tol, cg_max_iter, int(bool(compute_e3)), int(precond),
                        int(precision), float(inner_rel_tol))
        r = Result()
        self._ok(self.lib.mpspt_sweep(self.h, C.byref(p), C.byref(r)))
        out = {f: getattr(r, f) for f, _ in Result._fields_}
        out["e2_sweep"] = list(r.e2_sweep)[:r.n_sweeps_done]
        out["t_phase"] = dict(zip(("twoop", "build", "solve", "truncate", "env", "guess"), list(r.t_phase)))
        return out

    # learned preconditioner
    @staticmethod
    def _f32(a, shape=None):
        a = np.ascontiguousarray(a, dtype=np.float32)
        if shape is not None and a.shape != shape:
            raise ValueError(f"expected shape {shape}, got {a.shape}")
        return a, a.ctypes.data_as(C.POINTER(C.c_float))

    def precond_set(self, params):
        a, pa = self._f32(params)
        self._ok(self.lib.mpspt_precond_set(self.h, pa, a.size))

    def precond_get(self):
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        self._ok(self.lib.mpspt_precond_get(self.h, out.ctypes.data_as(C.POINTER(C.c_float)), out.size))
        return out

    def mlp_grad(self, X, t):
        Xa, px = self._f32(X)
        ta, pt = self._f32(t)
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = C.c_float()
        self._ok(self.lib.mpspt_mlp_grad(self.h, px, pt, ta.size, g.ctypes.data_as(C.POINTER(C.c_float)),
                                         C.byref(loss)))
        return loss.value, g

    def mlp_train_step(self, X, t, lr):
        Xa, px = self._f32(X)
        ta, pt = self._f32(t)
        loss = C.c_float()
        self._ok(self.lib.mpspt_mlp_train_step(self.h, px, pt, ta.size, lr, C.byref(loss)))
        return loss.value

    def harvest(self, enable=True):
        self._ok(self.lib.mpspt_harvest(self.h, int(bool(enable))))

    def harvest_get(self):
        n = C.c_int64()
        self._ok(self.lib.mpspt_harvest_get(self.h, 0, None, None, C.byref(n)))
        X = np.zeros((n.value, MLP_INPUTS), dtype=np.float32)
        t = np.zeros(n.value, dtype=np.float32)
        if n.value:
            self._ok(self.lib.mpspt_harvest_get(self.h, n.value, X.ctypes.data_as(C.POINTER(C.c_float)),
                                                t.ctypes.data_as(C.POINTER(C.c_float)), C.byref(n)))
        return X, t

    def set_tuning(self, wide_chunks, kseg_min, kseg_div, split_waves=4):
        self._ok(self.lib.mpspt_set_tuning(self.h, int(wide_chunks), int(kseg_min), int(kseg_div), int(split_waves)))

    def get_tuning(self):
        a, b, c, d = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        self._ok(self.lib.mpspt_get_tuning(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return {"wide_chunks": a.value, "kseg_min": b.value, "kseg_div": c.value, "split_waves": d.value}

    def profile(self, enable=True, every=1):
        """Record kernel durations (every ``every``-th launch of each kind), or stop."""
        self._ok(self.lib.mpspt_profile(self.h, int(every) if enable else 0))

    KERNELS = {0: "k_gemm_grouped", 1: "k_axpy_grouped", 2: "k_eig_reduce", 3: "k_diag_grouped", 4: "k_eig_vectors",
               5: "vector kernels", 6: "k_gemm_grouped_lo", 7: "k_axpy_grouped_lo"}

    def kernel_stats(self, kind):
        s, n, f, b, na = C.c_double(), C.c_int64(), C.c_double(), C.c_double(), C.c_int64()
        self._ok(self.lib.mpspt_kernel_stats(self.h, kind, C.byref(s), C.byref(n), C.byref(f), C.byref(b),
                                             C.byref(na)))
        return dict(kernel=self.KERNELS.get(kind, str(kind)), seconds=s.value, launches=n.value, flops=f.value,
                    bytes=b.value, launches_all=na.value)

    def get_trace(self):
        n = C.c_int32()
        self._ok(self.lib.mpspt_get_trace(self.h, 0, None, None, None, None, C.byref(n)))
        m = n.value
        e2, cg, disc, t = np.zeros(m), np.zeros(m, dtype=np.int32), np.zeros(m), np.zeros(m)
        self._ok(self.lib.mpspt_get_trace(self.h, m, e2.ctypes.data_as(C.POINTER(C.c_double)),
                                          cg.ctypes.data_as(C.POINTER(C.c_int32)),
                                          disc.ctypes.data_as(C.POINTER(C.c_double)),
                                          t.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)))
        return dict(e2=e2, cg_iters=cg, discarded=disc, t=t)

    def get_bond(self, which, bond):
        n = C.c_int32()
        buf = np.zeros(3 * 512, dtype=np.int32)
        self._ok(self.lib.mpspt_get_bond(self.h, which, bond, 512, buf.ctypes.data_as(C.POINTER(C.c_int32)),
                                         C.byref(n)))
        return [((int(buf[3 * i]), int(buf[3 * i + 1])), int(buf[3 * i + 2])) for i in range(n.value)]

    def get_site(self, which, site):
        dims = np.zeros(2, dtype=np.int32)
        self._ok(self.lib.mpspt_get_site(self.h, which, site, 0, None, dims.ctypes.data_as(C.POINTER(C.c_int32))))
        out = np.zeros((dims[0], 4, dims[1]))
        self._ok(self.lib.mpspt_get_site(self.h, which, site, out.size, out.ctypes.data_as(C.POINTER(C.c_double)),
                                         dims.ctypes.data_as(C.POINTER(C.c_int32))))
        return out


def mpo_dense(k_a, k_v, h, eri, eps_virt, which, lib=None):
    """Contract one of the library's MPOs to a dense matrix (host only, n <= 6)."""
    lib = lib or load_library()
    n = k_a + k_v
    out = np.zeros((4 ** n, 4 ** n))
    (h, hp), (e, ep), (v, vp) = _d(h), _d(eri), _d(eps_virt)
    st = lib.mpspt_mpo_dense(k_a, k_v, hp, ep, vp, which, out.ctypes.data_as(C.POINTER(C.c_double)), out.size)
    if st != 0:
        raise MPSPTError(st, lib.mpspt_last_error(None).decode())
    return out


def mpo_dims(k_a, k_v, h, eri, eps_virt, which, lib=None):
    lib = lib or load_library()
    n = k_a + k_v
    out = np.zeros(n + 1, dtype=np.int32)
    (h, hp), (e, ep), (v, vp) = _d(h), _d(eri), _d(eps_virt)
    st = lib.mpspt_mpo_dims(k_a, k_v, hp, ep, vp, which, out.ctypes.data_as(C.POINTER(C.c_int32)), n + 1)
    if st != 0:
        raise MPSPTError(st, lib.mpspt_last_error(None).decode())
    return out
