"""ctypes binding of libqdta.so (include/qdta.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Device arrays are torch tensors on the context's device (their
data_ptr() is passed); host arrays are numpy arrays.  The binding fails
loudly when the library has not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqdta.so")

OK, EARG, ECSR, EVAL, EUNREACH, EOVF, ENOMEM, EHIP, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7, -8
WABSORB = 1
RULE_NONE, RULE_CEIL, RULE_FLOOR, RULE_PROGRESS = 0, 1, 2, 3
LS_KSECTION, LS_QN, LS_MSA = 0, 1, 2
OBJ_UE, OBJ_SO = 0, 1
STOP_GAP, STOP_OBJ = 0, 1
FX = 1 << 20

EXPORTS = [
    "qdta_default_opts", "qdta_strerror", "qdta_last_error", "qdta_create", "qdta_destroy", "qdta_set_stream",
    "qdta_add_network", "qdta_set_demand", "qdta_layout", "qdta_offsets", "qdta_bpr", "qdta_trees", "qdta_aon",
    "qdta_get_legs", "qdta_ls_eval", "qdta_line_search", "qdta_fw_update", "qdta_solve", "qdta_get_flows",
    "qdta_get_costs", "qdta_advance_interval", "qdta_get_residual", "qdta_set_residual", "qdta_adjoint_record",
    "qdta_model_forward", "qdta_model_backward", "qdta_fw_begin", "qdta_fw_step",
    "qdta_profile_enable", "qdta_profile_read", "qdta_autotune", "qdta_workspace_query", "qdta_bind_workspace",
    "qdta_alloc_count", "qdta_ls_eval_noalloc",
]
PHASES = ["bpr", "sssp", "walk", "gap", "line_search", "update", "graph_iteration", "fill"]


class Opts(C.Structure):
    _fields_ = [("alpha", C.c_double), ("beta", C.c_int32), ("trunc_rule", C.c_int32), ("ls_mode", C.c_int32),
                ("K", C.c_int32), ("passes", C.c_int32), ("max_ls", C.c_int32), ("T1", C.c_double),
                ("T2", C.c_double), ("dx", C.c_double), ("stop_rule", C.c_int32), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("fixed_iters", C.c_int32), ("keep_history", C.c_int32),
                ("waves_per_cu", C.c_int32), ("delta_scale", C.c_double), ("sssp_shape", C.c_int32),
                ("launch_form", C.c_int32), ("tree_waves", C.c_int32), ("history_mib", C.c_int32),
                ("objective", C.c_int32), ("sssp_kernel", C.c_int32), ("load_form", C.c_int32),
                ("pad1", C.c_int32), ("progress_quantum_s", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("ls_evals", C.c_int32), ("qn_iters", C.c_int32), ("absorb", C.c_int32),
                ("stopped_by", C.c_int32), ("status", C.c_int32), ("gap", C.c_double), ("objective", C.c_double),
                ("last_alpha", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LayoutInfo(C.Structure):
    _fields_ = [("n_instances", C.c_int32), ("total_nodes", C.c_int64), ("total_links", C.c_int64),
                ("total_legs", C.c_int64), ("total_dests", C.c_int64)]


class Profile(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("count", C.c_int64 * 8), ("sssp_nodes", C.c_int64),
                ("sssp_links", C.c_int64)]


class QdtaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qdta error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run paper_2104_12911_amd/build.py (hipcc, gfx950)")
        # torch supplies the device memory and the streams, so the library must
        # run on torch's HIP runtime: load torch first, so that the runtime the
        # library links against (same soname) resolves to the one torch loaded
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.qdta_default_opts.argtypes = [vp]
        L.qdta_default_opts.restype = None
        L.qdta_strerror.argtypes = [C.c_int]
        L.qdta_strerror.restype = C.c_char_p
        L.qdta_last_error.argtypes = [vp]
        L.qdta_last_error.restype = C.c_char_p
        L.qdta_create.argtypes = [C.POINTER(vp), C.c_int, vp]
        L.qdta_destroy.argtypes = [vp]
        L.qdta_set_stream.argtypes = [vp, vp]
        L.qdta_add_network.argtypes = [vp, i32, i32, vp, vp, vp, vp, C.POINTER(i32)]
        L.qdta_set_demand.argtypes = [vp, i32, i32, vp, vp, vp, dbl]
        L.qdta_layout.argtypes = [vp, vp]
        L.qdta_offsets.argtypes = [vp, vp, vp, vp, vp]
        L.qdta_bpr.argtypes = [vp, vp, vp, vp]
        L.qdta_trees.argtypes = [vp, vp, i32, vp, i32, vp, vp, vp]
        L.qdta_aon.argtypes = [vp, vp, vp, vp, vp, vp]
        L.qdta_get_legs.argtypes = [vp, vp, vp, vp, vp]
        L.qdta_ls_eval.argtypes = [vp, vp, vp, vp, i32, vp, vp]
        L.qdta_ls_eval_noalloc.argtypes = [vp, vp, vp, vp, i32, vp, vp]
        L.qdta_line_search.argtypes = [vp, vp, vp, vp, i32, vp]
        L.qdta_fw_update.argtypes = [vp, vp, vp, vp]
        L.qdta_solve.argtypes = [vp, vp, vp]
        L.qdta_get_flows.argtypes = [vp, vp]
        L.qdta_get_costs.argtypes = [vp, vp, vp]
        L.qdta_advance_interval.argtypes = [vp, vp]
        L.qdta_get_residual.argtypes = [vp, i32, C.POINTER(i64), vp, vp, vp, C.POINTER(i64), vp]
        L.qdta_set_residual.argtypes = [vp, i32, i64, vp, vp, vp, vp]
        L.qdta_adjoint_record.argtypes = [vp, vp]
        L.qdta_model_forward.argtypes = [vp, vp, vp, vp, vp, C.POINTER(C.c_uint64)]
        L.qdta_model_backward.argtypes = [vp, C.c_uint64, vp, vp, vp]
        L.qdta_workspace_query.argtypes = [vp, vp, i64, i64, C.POINTER(C.c_size_t)]
        L.qdta_bind_workspace.argtypes = [vp, vp, C.c_size_t]
        L.qdta_alloc_count.argtypes = [vp, C.POINTER(i64), C.POINTER(C.c_size_t)]
        L.qdta_fw_begin.argtypes = [vp, vp]
        L.qdta_fw_step.argtypes = [vp, vp, vp, C.POINTER(i32)]
        L.qdta_profile_enable.argtypes = [vp, i32]
        L.qdta_profile_read.argtypes = [vp, vp]
        L.qdta_autotune.argtypes = [vp, vp, dbl, C.POINTER(dbl)]
        for name in EXPORTS:
            if name not in ("qdta_default_opts", "qdta_strerror", "qdta_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().qdta_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    """Pointer of a numpy array (host) or torch tensor (device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())


def _check_tensor(t, dtype, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != getattr(torch, dtype) or not t.is_contiguous() or t.numel() < numel:
        raise ValueError(f"{name}: need contiguous {dtype} with >= {numel} elements")


class Context:
    """One library context: a set of network instances, their demand and the
    Frank-Wolfe state, on one device and stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        rc = lib().qdta_create(C.byref(h), device, C.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise QdtaError(rc, lib().qdta_strerror(rc).decode())
        self._h = h
        self.n_inst = 0
        self._nets = []

    def close(self):
        if getattr(self, "_h", None):
            lib().qdta_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _rc(self, rc, allow=(OK,)):
        if rc in allow:
            return rc
        if rc > 0:
            return rc
        raise QdtaError(rc, lib().qdta_last_error(self._h).decode() or lib().qdta_strerror(rc).decode())

    # --- setup (host arrays) ------------------------------------------------
    def add_network(self, n, row_ptr, col, fftt, cap) -> int:
        rp, cl = _np(row_ptr, np.int32), _np(col, np.int32)
        ff, cp = _np(fftt, np.float32), _np(cap, np.float32)
        out = C.c_int32()
        self._rc(lib().qdta_add_network(self._h, int(n), int(cl.shape[0]), _ptr(rp), _ptr(cl), _ptr(ff), _ptr(cp),
                                        C.byref(out)))
        self.n_inst += 1
        self._nets.append((int(n), int(cl.shape[0])))
        return out.value

    def add(self, net) -> int:
        return self.add_network(net.n, net.row_ptr, net.col, net.fftt, net.cap)

    def set_demand(self, inst, orig, dest, trips, dt_s):
        o, d, t = _np(orig, np.int32), _np(dest, np.int32), _np(trips, np.float64)
        self._rc(lib().qdta_set_demand(self._h, int(inst), int(o.shape[0]), _ptr(o), _ptr(d), _ptr(t), float(dt_s)))

    def layout(self) -> LayoutInfo:
        li = LayoutInfo()
        self._rc(lib().qdta_layout(self._h, C.byref(li)))
        return li

    def offsets(self):
        k = self.n_inst + 1
        arrs = [np.zeros(k, np.int64) for _ in range(4)]
        self._rc(lib().qdta_offsets(self._h, *[_ptr(a) for a in arrs]))
        return dict(zip(["node", "link", "leg", "dest"], arrs))

    def legs(self, with_delay=False):
        """(orig, dest, d_fx) of the current legs; with_delay adds their carried delays."""
        P = self.layout().total_legs
        o, d, w = np.zeros(P, np.int32), np.zeros(P, np.int32), np.zeros(P, np.int64)
        t = np.zeros(P, np.float32)
        self._rc(lib().qdta_get_legs(self._h, _ptr(o), _ptr(d), _ptr(w), _ptr(t)))
        return (o, d, w, t) if with_delay else (o, d, w)

    # --- hot-path pieces (device tensors) ------------------------------------
    def bpr(self, opts, f_fx, cost):
        self._rc(lib().qdta_bpr(self._h, C.byref(opts), _ptr(f_fx), _ptr(cost)))

    def trees(self, opts, inst, cost, dest, dist, succ):
        return self._rc(lib().qdta_trees(self._h, C.byref(opts), int(inst), _ptr(cost), int(dest.numel()), _ptr(dest),
                                         _ptr(dist), _ptr(succ)), allow=(OK, WABSORB))

    def aon(self, opts, cost, y_fx, stop=None, stop_delay=None):
        return self._rc(lib().qdta_aon(self._h, C.byref(opts), _ptr(cost), _ptr(y_fx), _ptr(stop), _ptr(stop_delay)),
                        allow=(OK, WABSORB))

    def ls_eval(self, opts, f_fx, y_fx, alphas, sums):
        K = alphas.shape[-1]
        self._rc(lib().qdta_ls_eval(self._h, C.byref(opts), _ptr(f_fx), _ptr(y_fx), int(K), _ptr(alphas), _ptr(sums)))

    def ls_eval_noalloc(self, opts, f_fx, y_fx, alphas, sums):
        """ls_eval with its scratch in the library's static device array (no allocation)."""
        K = alphas.shape[-1]
        self._rc(lib().qdta_ls_eval_noalloc(self._h, C.byref(opts), _ptr(f_fx), _ptr(y_fx), int(K), _ptr(alphas),
                                            _ptr(sums)))

    def line_search(self, opts, f_fx, y_fx, j, alpha_out):
        self._rc(lib().qdta_line_search(self._h, C.byref(opts), _ptr(f_fx), _ptr(y_fx), int(j), _ptr(alpha_out)))

    def fw_update(self, f_fx, y_fx, alpha):
        self._rc(lib().qdta_fw_update(self._h, _ptr(f_fx), _ptr(y_fx), _ptr(alpha)))

    def solve(self, opts):
        st = (Stats * max(self.n_inst, 1))()
        rc = self._rc(lib().qdta_solve(self._h, C.byref(opts), st), allow=(OK, WABSORB))
        return [st[i].as_dict() for i in range(self.n_inst)], rc

    def fw_begin(self, opts):
        self._rc(lib().qdta_fw_begin(self._h, C.byref(opts)))

    def fw_step(self, opts):
        st = (Stats * max(self.n_inst, 1))()
        live = C.c_int32()
        self._rc(lib().qdta_fw_step(self._h, C.byref(opts), st, C.byref(live)), allow=(OK, WABSORB))
        return [st[i].as_dict() for i in range(self.n_inst)], bool(live.value)

    def autotune(self, opts, budget_ms=2000.0):
        """Fastest kernel shape and bucket width for the current demand; returns
        (tuned opts, best trial ms).  The given opts object is updated in place."""
        best = C.c_double()
        self._rc(lib().qdta_autotune(self._h, C.byref(opts), float(budget_ms), C.byref(best)))
        return opts, best.value

    def profile(self, on: bool = True):
        self._rc(lib().qdta_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        p = Profile()
        self._rc(lib().qdta_profile_read(self._h, C.byref(p)))
        out = {name: (p.ms[i], p.count[i]) for i, name in enumerate(PHASES)}
        out["sssp_work"] = (p.sssp_nodes, p.sssp_links)
        return out

    def get_flows(self, f_fx):
        self._rc(lib().qdta_get_flows(self._h, _ptr(f_fx)))

    def get_costs(self, opts, cost):
        self._rc(lib().qdta_get_costs(self._h, C.byref(opts), _ptr(cost)))

    def advance_interval(self, opts):
        return self._rc(lib().qdta_advance_interval(self._h, C.byref(opts)), allow=(OK, WABSORB))

    def residual(self, inst, with_delay=False):
        """(orig, dest, w_fx, done_fx) of the pending residual; with_delay:
        (orig, dest, w_fx, delay, done_fx)."""
        cnt, done = C.c_int64(), C.c_int64()
        self._rc(lib().qdta_get_residual(self._h, int(inst), C.byref(cnt), None, None, None, C.byref(done), None))
        k = cnt.value
        o, d, w = np.zeros(k, np.int32), np.zeros(k, np.int32), np.zeros(k, np.int64)
        t = np.zeros(k, np.float32)
        self._rc(lib().qdta_get_residual(self._h, int(inst), C.byref(cnt), _ptr(o), _ptr(d), _ptr(w), C.byref(done),
                                         _ptr(t)))
        return (o, d, w, t, done.value) if with_delay else (o, d, w, done.value)

    def adjoint_record(self, opts):
        return self._rc(lib().qdta_adjoint_record(self._h, C.byref(opts)))

    def model_forward(self, opts, d, cap, f_out):
        """Forward pass of the frozen-path model; returns its id (for model_backward)."""
        li = self.layout()
        _check_tensor(d, "float64", li.total_legs, "d")
        if cap is not None:
            _check_tensor(cap, "float32", li.total_links, "cap")
        _check_tensor(f_out, "float64", li.total_links, "f_out")
        fid = C.c_uint64(0)
        self._rc(lib().qdta_model_forward(self._h, C.byref(opts), _ptr(d), _ptr(cap), _ptr(f_out), C.byref(fid)))
        return fid.value

    def model_backward(self, fwd_id, fbar, dbar, capbar):
        li = self.layout()
        _check_tensor(fbar, "float64", li.total_links, "fbar")
        _check_tensor(dbar, "float64", li.total_legs, "dbar")
        _check_tensor(capbar, "float64", li.total_links, "capbar")
        return self._rc(lib().qdta_model_backward(self._h, int(fwd_id), _ptr(fbar), _ptr(dbar), _ptr(capbar)))

    def workspace_query(self, opts, max_legs=0, max_dests=0):
        """Bytes of device memory the context needs for its networks, the
        current demand (or max_legs / max_dests if larger) and opts."""
        b = C.c_size_t(0)
        self._rc(lib().qdta_workspace_query(self._h, C.byref(opts), int(max_legs), int(max_dests), C.byref(b)))
        return b.value

    def bind_workspace(self, ws):
        """Carve every device buffer from ws (a uint8 torch tensor the caller
        owns and keeps alive); the library then never calls hipMalloc."""
        if str(ws.dtype) != "torch.uint8" or not ws.is_cuda or not ws.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 CUDA tensor")
        self._ws = ws
        return self._rc(lib().qdta_bind_workspace(self._h, C.c_void_p(ws.data_ptr()), ws.numel()))

    def alloc_count(self):
        """(hipMalloc calls made by this context, workspace bytes in use)."""
        n, u = C.c_int64(0), C.c_size_t(0)
        self._rc(lib().qdta_alloc_count(self._h, C.byref(n), C.byref(u)))
        return n.value, u.value

    def set_residual(self, inst, orig, dest, w_fx, delay=None):
        o, d, w = _np(orig, np.int32), _np(dest, np.int32), _np(w_fx, np.int64)
        t = None if delay is None else _np(delay, np.float32)
        if not (len(o) == len(d) == len(w)) or (t is not None and len(t) != len(o)):
            raise ValueError("residual arrays differ in length")
        self._rc(lib().qdta_set_residual(self._h, int(inst), len(o), _ptr(o), _ptr(d), _ptr(w), _ptr(t)))


def _frozen_path_flows_class():
    import torch

    class FrozenPathFlows(torch.autograd.Function):
        """f = M(d, C): the link flows (veh) of a solved interval's Frank-Wolfe
        updates replayed on their frozen paths (qdta_model_forward), with the
        reverse pass of qdta_model_backward.  Needs Context.adjoint_record
        after the solve.  The context keeps the iterates of its last forward
        pass only: the backward of an earlier one raises (QDTA_ESTATE)
        instead of returning another pass's gradients."""

        @staticmethod
        def forward(ctx, qctx, opts, d, cap):
            li = qctx.layout()
            f = torch.empty(li.total_links, dtype=torch.float64, device=d.device)
            ctx.fwd_id = qctx.model_forward(opts, d.detach().contiguous(),
                                            None if cap is None else cap.detach().contiguous(), f)
            ctx.qctx = qctx
            ctx.cap_dtype = None if cap is None else cap.dtype
            return f

        @staticmethod
        def backward(ctx, fbar):
            qctx = ctx.qctx
            li = qctx.layout()
            dbar = torch.empty(li.total_legs, dtype=torch.float64, device=fbar.device)
            capbar = torch.empty(li.total_links, dtype=torch.float64, device=fbar.device)
            qctx.model_backward(ctx.fwd_id, fbar.to(torch.float64).contiguous(), dbar, capbar)
            return None, None, dbar, (None if ctx.cap_dtype is None else capbar.to(ctx.cap_dtype))

    return FrozenPathFlows


_FPF = None


def frozen_path_flows(qctx, opts, d, cap=None):
    """Differentiable link flows of the frozen-path model (see FrozenPathFlows)."""
    global _FPF
    if _FPF is None:
        _FPF = _frozen_path_flows_class()
    return _FPF.apply(qctx, opts, d, cap)
