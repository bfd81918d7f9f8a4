"""ctypes binding of the C ABI in ``include/eqs.h`` (argument marshalling only).

Every numerical step runs in the HIP library ``libeqs.so``; this module only
converts arguments. Device vectors are passed as torch CUDA (HIP) tensors of
dtype float64 (their ``data_ptr()`` is handed to the library) or as raw
integer device addresses. If the library is missing the import fails loudly:
there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeqs.so")

EQS_OK = 0
EQS_ERR_INVALID_ARG = -1
EQS_ERR_STATE = -2
EQS_ERR_HIP = -3
EQS_ERR_NOT_CONVERGED = -4
EQS_ERR_BREAKDOWN = -5
EQS_ERR_NONFINITE = -6
EQS_ERR_ALLOC = -7
EQS_MAX_DRIVES = 65536
EQS_MAX_GRAPH_ITERS = 256
EQS_PREC_FP64 = 0
EQS_PREC_FP32 = 1

ERROR_NAMES = {
    EQS_ERR_INVALID_ARG: "EQS_ERR_INVALID_ARG",
    EQS_ERR_STATE: "EQS_ERR_STATE",
    EQS_ERR_HIP: "EQS_ERR_HIP",
    EQS_ERR_NOT_CONVERGED: "EQS_ERR_NOT_CONVERGED",
    EQS_ERR_BREAKDOWN: "EQS_ERR_BREAKDOWN",
    EQS_ERR_NONFINITE: "EQS_ERR_NONFINITE",
    EQS_ERR_ALLOC: "EQS_ERR_ALLOC",
}


class eqs_material(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("kappa0", C.c_double), ("e_s", C.c_double), ("alpha", C.c_double),
                ("nonlinear", C.c_int32), ("reserved", C.c_int32)]


class eqs_drive(C.Structure):
    _fields_ = [("amp", C.c_double), ("freq", C.c_double), ("phase", C.c_double)]


class eqs_amg_params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("coarse_max", C.c_int32), ("max_levels", C.c_int32),
                ("flexible", C.c_int32), ("theta", C.c_double), ("jacobi_weight", C.c_double),
                ("smooth_weight", C.c_double)]


class eqs_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("relres", C.c_double)]


class eqs_step_stats(C.Structure):
    _fields_ = [("stages", C.c_int32), ("total_iters", C.c_int32), ("max_iters", C.c_int32),
                ("min_iters", C.c_int32), ("not_converged", C.c_int32), ("guess_used", C.c_int32),
                ("guess_fallbacks", C.c_int32), ("reserved", C.c_int32), ("max_relres", C.c_double),
                ("train_loss", C.c_double)]


class eqs_guess_params(C.Structure):
    _fields_ = [("kind", C.c_int32), ("window", C.c_int32), ("capacity", C.c_int32), ("warmup", C.c_int32),
                ("batch", C.c_int32), ("bf16", C.c_int32), ("guard", C.c_int32), ("add_threshold", C.c_int32),
                ("lr", C.c_double), ("seed", C.c_uint64), ("init", C.c_void_p)]


EQS_GUESS_PREVIOUS = 0
EQS_GUESS_ZERO = 1
EQS_GUESS_GALERKIN = 2
EQS_GUESS_MLP = 3
EQS_GUESS_MOR = 4
EQS_MLP_NPARAM = 7312
GUESS_KINDS = {"previous": EQS_GUESS_PREVIOUS, "zero": EQS_GUESS_ZERO, "galerkin": EQS_GUESS_GALERKIN,
               "mlp": EQS_GUESS_MLP, "mor": EQS_GUESS_MOR}


class eqs_adapt_params(C.Structure):
    _fields_ = [("atol", C.c_double), ("rtol", C.c_double), ("tau0", C.c_double), ("tau_min", C.c_double),
                ("tau_max", C.c_double), ("s_max", C.c_int32), ("max_attempts", C.c_int32)]


class eqs_adapt_record(C.Structure):
    _fields_ = [("t", C.c_double), ("tau", C.c_double), ("err", C.c_double), ("s", C.c_int32),
                ("accepted", C.c_int32)]


class eqs_adapt_stats(C.Structure):
    _fields_ = [("accepted", C.c_int32), ("rejected", C.c_int32), ("max_s", C.c_int32), ("not_converged", C.c_int32),
                ("stages", C.c_int64), ("cg_iters", C.c_int64), ("last_tau", C.c_double)]


class eqs_info(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_tets", C.c_int64), ("n_free", C.c_int64), ("nnz_M", C.c_int64),
                ("n_levels", C.c_int32), ("precision", C.c_int32), ("level_rows", C.c_int64 * 16),
                ("level_nnz", C.c_int64 * 16), ("level_p_nnz", C.c_int64 * 16), ("level_r_nnz", C.c_int64 * 16),
                ("device_bytes", C.c_int64), ("workspace_bytes", C.c_int64), ("workspace_used", C.c_int64)]


_P = C.c_void_p
_SIGNATURES = {
    "eqs_create": ([C.POINTER(_P), C.c_int, _P], C.c_int),
    "eqs_destroy": ([_P], C.c_int),
    "eqs_set_mesh": ([_P, C.c_int64, _P, C.c_int64, _P], C.c_int),
    "eqs_set_mesh_p2": ([_P, C.c_int64, _P, C.c_int64, _P], C.c_int),
    "eqs_set_materials": ([_P, C.c_int32, _P, _P], C.c_int),
    "eqs_set_dirichlet": ([_P, C.c_int64, _P, _P, C.c_int32, _P], C.c_int),
    "eqs_build_preconditioner": ([_P, _P], C.c_int),
    "eqs_set_graph_iters": ([_P, C.c_int32], C.c_int),
    "eqs_set_deterministic": ([_P, C.c_int32], C.c_int),
    "eqs_state_size": ([_P, C.POINTER(C.c_int64)], C.c_int),
    "eqs_state_save": ([_P, _P, C.c_int64], C.c_int),
    "eqs_state_load": ([_P, _P, C.c_int64], C.c_int),
    "eqs_get_info": ([_P, _P], C.c_int),
    "eqs_query": ([_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "eqs_set_workspace": ([_P, _P, C.c_int64], C.c_int),
    "eqs_apply_K": ([_P, C.c_double, _P, _P], C.c_int),
    "eqs_stage_rhs": ([_P, C.c_double, _P, _P], C.c_int),
    "eqs_apply_M": ([_P, _P, _P], C.c_int),
    "eqs_apply_preconditioner": ([_P, _P, _P], C.c_int),
    "eqs_solve_M": ([_P, _P, _P, C.c_double, C.c_int32, _P], C.c_int),
    "eqs_rkc_step": ([_P, C.c_double, C.c_double, C.c_int32, _P, C.c_double, C.c_int32, _P], C.c_int),
    "eqs_rkc_adaptive": ([_P, C.c_double, C.c_double, _P, C.c_double, C.c_int32, _P, _P, C.c_int32,
                          C.POINTER(C.c_int32), _P], C.c_int),
    "eqs_set_guess": ([_P, _P], C.c_int),
    "eqs_galerkin_start": ([_P, C.c_int32, _P, _P, _P, _P, C.POINTER(C.c_int32)], C.c_int),
    "eqs_galerkin_start_noalloc": ([_P, C.c_int32, _P, _P, _P, _P, C.POINTER(C.c_int32)], C.c_int),
    "eqs_set_instances": ([_P, C.c_int32, _P, _P], C.c_int),
    "eqs_instance_stats": ([_P, C.c_int32, _P, _P], C.c_int),
    "eqs_stage_iters": ([_P, _P, C.c_int32, _P], C.c_int),
    "eqs_batch_create": ([C.POINTER(_P), C.c_int32, _P, C.c_int, _P, _P], C.c_int),
    "eqs_batch_destroy": ([_P], C.c_int),
    "eqs_batch_set_graph_iters": ([_P, C.c_int32], C.c_int),
    "eqs_batch_rkc_steps": ([_P, C.c_int32, C.c_double, C.c_double, C.c_int32, _P, C.c_double, C.c_int32, _P],
                            C.c_int),
    "eqs_batch_instance_stats": ([_P, _P, _P], C.c_int),
    "eqs_mlp_create": ([C.POINTER(_P), C.c_int, _P, _P, C.c_int32, C.c_double], C.c_int),
    "eqs_mlp_destroy": ([_P], C.c_int),
    "eqs_mlp_forward": ([_P, _P, _P, C.c_int32], C.c_int),
    "eqs_mlp_train_step": ([_P, _P, _P, C.c_int32, C.POINTER(C.c_float)], C.c_int),
    "eqs_mlp_get": ([_P, _P, _P], C.c_int),
    "eqs_profile_enable": ([_P, C.c_uint32], C.c_int),
    "eqs_profile_read": ([_P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)], C.c_int),
    "eqs_describe": ([_P, C.c_char_p, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
    "eqs_last_error": ([], C.c_char_p),
}

KCLASS = {
    "element": 0,
    "spmv_M": 1,
    "presmooth0": 2,
    "postsmooth0": 3,
    "vcycle": 4,
    "cg_update": 5,
    "rkc_combine": 6,
    "restrict0": 7,
    "prolong0": 8,
    "vcoarse": 9,
    "finalise": 10,
    "postsmooth1": 11,
}

_lib = None


def lib():
    """Load ``libeqs.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'` (no CPU fallback exists)"
            )
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class EqsError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().eqs_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {msg}")


def _check(code, where, ok=(EQS_OK,)):
    if code not in ok:
        raise EqsError(code, where)
    return code


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(_P)


def _dev(t, dtype="float64"):
    """Device address of a torch tensor (contiguous, given dtype) or an int address."""
    if isinstance(t, int):
        return _P(t)
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor on the GPU or an integer device address")
    if t.device.type != "cuda":
        raise ValueError("device vectors must live on the GPU")
    if t.dtype != getattr(torch, dtype) or not t.is_contiguous():
        raise ValueError(f"device vectors must be contiguous {dtype}")
    return _P(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return _P(stream)
    return _P(stream.cuda_stream)


class Context:
    """One EQS instance on one device (wraps ``eqs_ctx``)."""

    def __init__(self, device: int = 0, stream=None):
        self._h = _P()
        _check(lib().eqs_create(C.byref(self._h), device, _stream_handle(stream)), "eqs_create")
        self.device = device

    def close(self):
        if self._h:
            lib().eqs_destroy(self._h)
            self._h = _P()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- set-up ----------------------------------------------------------
    def set_mesh(self, xyz, tets):
        """4-node tets (n_tets x 4) or second-order 10-node tets (n_tets x 10)."""
        xyz, pxyz = _host(xyz, np.float64)
        tets, ptets = _host(tets, np.int32)
        if tets.ndim != 2 or tets.shape[1] not in (4, 10):
            raise ValueError("tets must be n_tets x 4 or n_tets x 10")
        fn, name = (lib().eqs_set_mesh_p2, "eqs_set_mesh_p2") if tets.shape[1] == 10 else (lib().eqs_set_mesh,
                                                                                           "eqs_set_mesh")
        _check(fn(self._h, xyz.shape[0], pxyz, tets.shape[0], ptets), name)

    def set_materials(self, eps_r, kappa0, e_s, alpha, nonlinear, tet_mat):
        n = len(eps_r)
        arr = (eqs_material * n)()
        for m in range(n):
            arr[m] = eqs_material(float(eps_r[m]), float(kappa0[m]), float(e_s[m]), float(alpha[m]),
                                  int(nonlinear[m]), 0)
        tm, ptm = _host(tet_mat, np.int32)
        _check(lib().eqs_set_materials(self._h, n, C.cast(arr, _P), ptm), "eqs_set_materials")

    def set_dirichlet(self, nodes, drive_id, amp, freq, phase):
        nodes, pn = _host(nodes, np.int32)
        did, pd = _host(drive_id, np.int32)
        n_drive = len(amp)
        arr = (eqs_drive * n_drive)()
        for k in range(n_drive):
            arr[k] = eqs_drive(float(amp[k]), float(freq[k]), float(phase[k]))
        _check(lib().eqs_set_dirichlet(self._h, nodes.shape[0], pn, pd, n_drive, C.cast(arr, _P)),
               "eqs_set_dirichlet")

    def build_preconditioner(self, precision=EQS_PREC_FP64, **kw):
        p = eqs_amg_params()
        p.precision = precision
        for k, v in kw.items():
            setattr(p, k, v)
        _check(lib().eqs_build_preconditioner(self._h, C.byref(p)), "eqs_build_preconditioner")

    def set_graph_iters(self, iters):
        """CG iterations replayed per captured graph launch (1 .. EQS_MAX_GRAPH_ITERS)."""
        _check(lib().eqs_set_graph_iters(self._h, int(iters)), "eqs_set_graph_iters")

    def state_save(self) -> bytes:
        """Checkpoint of the context's run state (eqs_state_save) as bytes."""
        n = C.c_int64(0)
        _check(lib().eqs_state_size(self._h, C.byref(n)), "eqs_state_size")
        buf = (C.c_char * max(1, n.value))()
        _check(lib().eqs_state_save(self._h, C.cast(buf, _P), n.value), "eqs_state_save")
        return bytes(buf[: n.value])

    def state_load(self, data: bytes):
        """Restore a checkpoint written by state_save (eqs_state_load)."""
        buf = C.create_string_buffer(bytes(data), max(1, len(data)))
        _check(lib().eqs_state_load(self._h, C.cast(buf, _P), len(data)), "eqs_state_load")

    def set_deterministic(self, on=True):
        """Element pass summed in a fixed order (bitwise reproducible); before the build."""
        _check(lib().eqs_set_deterministic(self._h, 1 if on else 0), "eqs_set_deterministic")

    def setup_case(self, case, precision=None, deterministic=None, **amg):
        """Hand a ``eqsgen.Case`` to the library (mesh, materials, Dirichlet, AMG)."""
        if deterministic is not None:
            self.set_deterministic(deterministic)
        self.set_mesh(case.xyz, case.tets)
        self.set_materials(case.eps_r, case.kappa0, case.e_s, case.alpha, case.nonlinear, case.tet_mat)
        self.set_dirichlet(case.dir_nodes, case.dir_drive, case.amp, case.freq, case.phase)
        if precision is None:
            precision = EQS_PREC_FP32 if case.precision == "fp32" else EQS_PREC_FP64
        self.build_preconditioner(precision, **amg)
        return self.info()

    def set_instances(self, node_off, tet_off):
        """Declare the mesh a concatenation of independent instances (batched form)."""
        no, pno = _host(node_off, np.int64)
        to, pto = _host(tet_off, np.int64)
        _check(lib().eqs_set_instances(self._h, no.size - 1, pno, pto), "eqs_set_instances")

    def instance_stats(self, n_inst):
        it = np.zeros(n_inst, np.int64)
        rr = np.zeros(n_inst)
        _check(lib().eqs_instance_stats(self._h, n_inst, it.ctypes.data_as(_P), rr.ctypes.data_as(_P)),
               "eqs_instance_stats")
        return it, rr

    def set_inputs(self, case):
        """Mesh, materials and Dirichlet data of a ``eqsgen.Case`` (no build)."""
        self.set_mesh(case.xyz, case.tets)
        self.set_materials(case.eps_r, case.kappa0, case.e_s, case.alpha, case.nonlinear, case.tet_mat)
        self.set_dirichlet(case.dir_nodes, case.dir_drive, case.amp, case.freq, case.phase)

    def info(self) -> dict:
        o = eqs_info()
        _check(lib().eqs_get_info(self._h, C.byref(o)), "eqs_get_info")
        L = o.n_levels
        return dict(n_nodes=o.n_nodes, n_tets=o.n_tets, n_free=o.n_free, nnz_M=o.nnz_M, n_levels=L,
                    precision=o.precision, level_rows=list(o.level_rows[:L]), level_nnz=list(o.level_nnz[:L]),
                    level_p_nnz=list(o.level_p_nnz[:L]), level_r_nnz=list(o.level_r_nnz[:L]),
                    device_bytes=o.device_bytes, workspace_bytes=o.workspace_bytes,
                    workspace_used=o.workspace_used)

    def query(self):
        """(n_free, ws_bytes): free nodes and the workspace size the context needs now."""
        nf, ws = C.c_int64(), C.c_int64()
        _check(lib().eqs_query(self._h, C.byref(nf), C.byref(ws)), "eqs_query")
        return nf.value, ws.value

    def set_workspace(self, ws=None):
        """Hand the context its device memory: a torch uint8 tensor on the
        context's device (kept referenced here while attached), or None to
        return to memory the library allocates."""
        if ws is None:
            _check(lib().eqs_set_workspace(self._h, None, 0), "eqs_set_workspace")
        else:
            if ws.device.type != "cuda" or not ws.is_contiguous():
                raise ValueError("the workspace must be a contiguous tensor on the GPU")
            _check(lib().eqs_set_workspace(self._h, _P(ws.data_ptr()), ws.numel() * ws.element_size()),
                   "eqs_set_workspace")
        self._ws = ws

    def use_torch_workspace(self, extra=0):
        """Allocate the workspace eqs_query asks for (plus `extra` bytes) with
        torch and attach it; returns the tensor."""
        import torch

        _, need = self.query()
        ws = torch.empty(need + extra, dtype=torch.uint8, device=torch.device("cuda", self.device))
        self.set_workspace(ws)
        return ws

    def describe(self) -> str:
        need = C.c_int64()
        _check(lib().eqs_describe(self._h, None, 0, C.byref(need)), "eqs_describe")
        buf = C.create_string_buffer(need.value)
        _check(lib().eqs_describe(self._h, buf, need.value, None), "eqs_describe")
        return buf.value.decode()

    # ---- per-kernel timing -----------------------------------------------
    def profile_enable(self, classes=()):
        """Time every launch of the named kernel classes with HIP events (resets counters)."""
        mask = 0
        for k in classes:
            mask |= 1 << KCLASS[k]
        _check(lib().eqs_profile_enable(self._h, mask), "eqs_profile_enable")

    def profile_read(self, kclass):
        n = C.c_int64()
        ms = C.c_double()
        _check(lib().eqs_profile_read(self._h, KCLASS[kclass], C.byref(n), C.byref(ms)), "eqs_profile_read")
        return dict(launches=n.value, total_ms=ms.value, avg_ms=ms.value / n.value if n.value else 0.0)

    # ---- hot path --------------------------------------------------------
    def apply_K(self, t, x, y):
        _check(lib().eqs_apply_K(self._h, float(t), _dev(x), _dev(y)), "eqs_apply_K")

    def stage_rhs(self, t, y_free, r):
        _check(lib().eqs_stage_rhs(self._h, float(t), _dev(y_free), _dev(r)), "eqs_stage_rhs")

    def apply_M(self, x, y):
        _check(lib().eqs_apply_M(self._h, _dev(x), _dev(y)), "eqs_apply_M")

    def apply_preconditioner(self, r, z):
        _check(lib().eqs_apply_preconditioner(self._h, _dev(r), _dev(z)), "eqs_apply_preconditioner")

    def solve_M(self, rhs, y, rtol, maxit=1000, allow_not_converged=False):
        st = eqs_solve_stats()
        ok = (EQS_OK, EQS_ERR_NOT_CONVERGED) if allow_not_converged else (EQS_OK,)
        rc = lib().eqs_solve_M(self._h, _dev(rhs), _dev(y), float(rtol), int(maxit), C.byref(st))
        _check(rc, "eqs_solve_M", ok)
        return dict(iters=st.iters, status=st.status, relres=st.relres, rc=rc)

    def rkc_step(self, t, dt, s, x, rtol, maxit=1000, allow_not_converged=False):
        st = eqs_step_stats()
        ok = (EQS_OK, EQS_ERR_NOT_CONVERGED) if allow_not_converged else (EQS_OK,)
        rc = lib().eqs_rkc_step(self._h, float(t), float(dt), int(s), _dev(x), float(rtol), int(maxit), C.byref(st))
        _check(rc, "eqs_rkc_step", ok)
        return dict(stages=st.stages, total_iters=st.total_iters, max_iters=st.max_iters, min_iters=st.min_iters,
                    not_converged=st.not_converged, guess_used=st.guess_used, guess_fallbacks=st.guess_fallbacks,
                    max_relres=st.max_relres, train_loss=st.train_loss, stage_iters=self.stage_iters(), rc=rc)

    def stage_iters(self):
        """CG iterations of each stage of the last rkc_step (eqs_stage_iters)."""
        buf = np.zeros(256, np.int32)
        n = C.c_int32(0)
        _check(lib().eqs_stage_iters(self._h, buf.ctypes.data_as(_P), buf.size, C.byref(n)), "eqs_stage_iters")
        return buf[:min(n.value, buf.size)].tolist()

    def rkc_adaptive(self, t0, t_end, x, rtol, atol_err, rtol_err, tau0, maxit=1000, s_max=0, tau_min=0.0,
                     tau_max=0.0, max_attempts=0, cap=100000, allow_not_converged=False):
        """Error-controlled RKC from t0 to t_end (eqs_rkc_adaptive); returns the
        stats and the list of attempted steps (t, tau, s, err, accepted)."""
        p = eqs_adapt_params(float(atol_err), float(rtol_err), float(tau0), float(tau_min), float(tau_max),
                             int(s_max), int(max_attempts))
        recs = (eqs_adapt_record * cap)()
        n = C.c_int32(0)
        st = eqs_adapt_stats()
        ok = (EQS_OK, EQS_ERR_NOT_CONVERGED) if allow_not_converged else (EQS_OK,)
        rc = lib().eqs_rkc_adaptive(self._h, float(t0), float(t_end), _dev(x), float(rtol), int(maxit), C.byref(p),
                                    C.cast(recs, _P), cap, C.byref(n), C.byref(st))
        _check(rc, "eqs_rkc_adaptive", ok)
        steps = [dict(t=recs[k].t, tau=recs[k].tau, s=recs[k].s, err=recs[k].err, accepted=bool(recs[k].accepted))
                 for k in range(min(n.value, cap))]
        return dict(accepted=st.accepted, rejected=st.rejected, max_s=st.max_s, not_converged=st.not_converged,
                    stages=st.stages, cg_iters=st.cg_iters, last_tau=st.last_tau, rc=rc), steps

    def set_guess(self, kind="previous", init=None, **kw):
        """Select the stage start vector: previous, zero, galerkin (eq. (5) on a sliding
        window), mor (eq. (5) on a fixed basis) or mlp."""
        p = eqs_guess_params()
        p.kind = GUESS_KINDS[kind] if isinstance(kind, str) else int(kind)
        p.bf16 = 1
        p.guard = 1
        p.warmup = 64
        for k, v in kw.items():
            setattr(p, k, v)
        keep = None
        if init is not None:
            keep = _flat_params(init)
            p.init = keep.ctypes.data_as(_P)
        _check(lib().eqs_set_guess(self._h, C.byref(p)), "eqs_set_guess")

    def galerkin_start(self, S, R, r, x0):
        """Eq. (5) on the window S (k x n_free, oldest first) with R = M S; writes
        x0 and returns the number of POD directions kept."""
        nf = self.info()["n_free"]
        if S.dim() != 2 or tuple(R.shape) != tuple(S.shape) or S.shape[1] != nf or r.numel() != nf or x0.numel() != nf:
            raise ValueError(f"galerkin_start: S and R must be k x {nf}, r and x0 hold {nf} values")
        m = C.c_int32(0)
        _check(lib().eqs_galerkin_start(self._h, int(S.shape[0]), _dev(S), _dev(R), _dev(r), _dev(x0), C.byref(m)),
               "eqs_galerkin_start")
        return int(m.value)


    def galerkin_start_noalloc(self, S, R, r, x0):
        """As galerkin_start, through eqs_galerkin_start_noalloc (no device
        allocation: the library's static scratch)."""
        nf = self.info()["n_free"]
        if S.dim() != 2 or tuple(R.shape) != tuple(S.shape) or S.shape[1] != nf or r.numel() != nf or x0.numel() != nf:
            raise ValueError(f"galerkin_start_noalloc: S and R must be k x {nf}, r and x0 hold {nf} values")
        m = C.c_int32(0)
        _check(lib().eqs_galerkin_start_noalloc(self._h, int(S.shape[0]), _dev(S), _dev(R), _dev(r), _dev(x0),
                                                C.byref(m)), "eqs_galerkin_start_noalloc")
        return int(m.value)


def _flat_params(params):
    """Concatenate {W1, b1, W2, b2, W3, b3} (or an already flat array) into float32."""
    if isinstance(params, dict):
        arr = np.concatenate([np.asarray(params[k], np.float32).reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])
    else:
        arr = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    if arr.size != EQS_MLP_NPARAM:
        raise ValueError(f"expected {EQS_MLP_NPARAM} parameters, got {arr.size}")
    return np.ascontiguousarray(arr)


def unflatten_params(flat):
    flat = np.asarray(flat)
    out, o = {}, 0
    for k, shp in (("W1", (64, 32)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (16, 64)), ("b3", (16,))):
        n = int(np.prod(shp))
        out[k] = flat[o:o + n].reshape(shp)
        o += n
    return out


class Mlp:
    """The start-vector network on its own (eqs_mlp_*): forward, train step, parameters."""

    def __init__(self, params, bf16=True, lr=1e-3, device=0, stream=None):
        self._h = _P()
        flat = _flat_params(params)
        _check(lib().eqs_mlp_create(C.byref(self._h), device, _stream_handle(stream), flat.ctypes.data_as(_P),
                                    1 if bf16 else 0, float(lr)), "eqs_mlp_create")

    def close(self):
        if self._h:
            lib().eqs_mlp_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, x, y):
        _check(lib().eqs_mlp_forward(self._h, _dev(x, "float32"), _dev(y, "float32"), int(x.shape[0])),
               "eqs_mlp_forward")

    def train_step(self, x, t):
        loss = C.c_float()
        _check(lib().eqs_mlp_train_step(self._h, _dev(x, "float32"), _dev(t, "float32"), int(x.shape[0]),
                                        C.byref(loss)), "eqs_mlp_train_step")
        return float(loss.value)

    def get(self):
        p = np.zeros(EQS_MLP_NPARAM, np.float32)
        g = np.zeros(EQS_MLP_NPARAM, np.float32)
        _check(lib().eqs_mlp_get(self._h, p.ctypes.data_as(_P), g.ctypes.data_as(_P)), "eqs_mlp_get")
        return unflatten_params(p), unflatten_params(g)


class Batch:
    """Independent instances advanced together (eqs_batch_*)."""

    def __init__(self, contexts, precision=EQS_PREC_FP64, device=0, stream=None, **amg):
        self._h = _P()
        self.n = len(contexts)
        arr = (_P * self.n)(*[c._h for c in contexts])
        p = eqs_amg_params()
        p.precision = precision
        for k, v in amg.items():
            setattr(p, k, v)
        _check(lib().eqs_batch_create(C.byref(self._h), self.n, C.cast(arr, _P), device, _stream_handle(stream),
                                      C.byref(p)), "eqs_batch_create")

    def close(self):
        if self._h:
            lib().eqs_batch_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph_iters(self, iters):
        """CG iterations replayed per captured graph launch (1 .. EQS_MAX_GRAPH_ITERS)."""
        _check(lib().eqs_batch_set_graph_iters(self._h, int(iters)), "eqs_batch_set_graph_iters")

    def rkc_steps(self, nsteps, t0, dt, s, xs, rtol, maxit=1000):
        ptrs = (_P * self.n)(*[_dev(x) for x in xs])
        st = eqs_step_stats()
        _check(lib().eqs_batch_rkc_steps(self._h, int(nsteps), float(t0), float(dt), int(s), C.cast(ptrs, _P),
                                         float(rtol), int(maxit), C.byref(st)), "eqs_batch_rkc_steps")
        it = np.zeros(self.n, np.int64)
        rr = np.zeros(self.n)
        _check(lib().eqs_batch_instance_stats(self._h, it.ctypes.data_as(_P), rr.ctypes.data_as(_P)),
               "eqs_batch_instance_stats")
        return dict(iters=it, relres=rr, last_step_total_iters=st.total_iters)
