"""Thin Python binding of libdcflow.so (argument marshalling only).

Every step of the screen runs in the library's HIP kernels; PyTorch provides
device memory (the workspace, batch, flow and score buffers) and the stream.
The entry points keep the C names: build_ptdf, eval_topologies,
eval_injections, n1_score.  There is no CPU fallback: if the shared library is
missing or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcflow.so")

DCFLOW_FP64 = 0
DCFLOW_FP32 = 1
PREC = {"fp64": DCFLOW_FP64, "fp32": DCFLOW_FP32, "bf16": 2, "bf16x6": 3}

ST_DISCONNECTED = 0x1
ST_SINGULAR = 0x2
ST_NONFINITE = 0x4
ST_ISLAND_SHIFT = 8

SCORE_DTYPE = np.dtype([("max_load", "<f8"), ("overload_sum", "<f8"), ("best_variant", "<i4"),
                        ("worst_branch", "<i4"), ("worst_outage", "<i4"), ("status", "<u4")])
CASE_DTYPE = np.dtype([("load", "<f8"), ("branch", "<i4"), ("outage", "<i4")])
WORST_MAX = 16


class DcflowError(RuntimeError):
    def __init__(self, code, what, bad_index=None):
        self.code = code
        self.bad_index = bad_index
        msg = f"{what}: {_lib.dcflow_strerror(code).decode()} ({code})"
        if bad_index is not None:
            msg += f", bad index {bad_index}"
        super().__init__(msg)


class GridDesc(ctypes.Structure):
    _fields_ = [("n_bus", ctypes.c_int32), ("n_branch", ctypes.c_int32), ("slack", ctypes.c_int32),
                ("from_", ctypes.c_void_p), ("to", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("n_mon", ctypes.c_int32), ("mon", ctypes.c_void_p),
                ("n_out", ctypes.c_int32), ("out", ctypes.c_void_p),
                ("p_base", ctypes.c_void_p), ("rating", ctypes.c_void_p),
                ("rating_scale", ctypes.c_double), ("rating_offset", ctypes.c_double),
                ("n_pst", ctypes.c_int32), ("pst_branch", ctypes.c_void_p),
                ("pst_scale", ctypes.c_double), ("n_hvdc", ctypes.c_int32),
                ("hvdc_from", ctypes.c_void_p), ("hvdc_to", ctypes.c_void_p),
                ("hvdc_scale", ctypes.c_double), ("n_gen_out", ctypes.c_int32),
                ("gen_bus", ctypes.c_void_p), ("gen_p", ctypes.c_void_p),
                ("n_multi_out", ctypes.c_int32), ("multi_off", ctypes.c_void_p),
                ("multi_br", ctypes.c_void_p)]


class Cands(ctypes.Structure):
    _fields_ = [("n_cand", ctypes.c_int32), ("off", ctypes.c_void_p), ("kind", ctypes.c_void_p),
                ("id", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("p_new", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    """dcflow_tuning: launch shapes of the N-1 scan (0 = automatic)."""
    _fields_ = [("scan_vc", ctypes.c_int32), ("scan_rchunk", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("scan_band", ctypes.c_int32),
                ("step_chunks", ctypes.c_int32), ("worst_record", ctypes.c_int32),
                ("guard_tol", ctypes.c_double)]

    def as_dict(self):
        d = {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "guard_tol"}
        d["guard_tol"] = float(self.guard_tol)
        return d


class PlanView(ctypes.Structure):
    _fields_ = [("n_bus", ctypes.c_int32), ("n_branch", ctypes.c_int32), ("n_mon", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("n_er", ctypes.c_int32), ("ld_h", ctypes.c_int32),
                ("ld_o", ctypes.c_int32), ("ptdf", ctypes.c_void_p), ("hdo", ctypes.c_void_p),
                ("f_base", ctypes.c_void_p), ("rating", ctypes.c_void_p), ("er", ctypes.c_void_p),
                ("n_inj", ctypes.c_int32), ("n_gen_out", ctypes.c_int32),
                ("n_multi_out", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2501_17529_amd.build_lib")
    # torch first: its HIP runtime (same soname as the one the library links) must
    # be the one loaded, since device pointers and streams come from torch
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    sig = {
        "dcflow_plan_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(SZ)]),
        "dcflow_build_ptdf": (ctypes.c_int, [P, P, SZ, P, ctypes.POINTER(P)]),
        "dcflow_plan_view_get": (ctypes.c_int, [P, P]),
        "dcflow_plan_destroy": (None, [P]),
        "dcflow_validate_candidates": (ctypes.c_int, [P, P, ctypes.POINTER(I32),
                                                      ctypes.POINTER(ctypes.c_int64),
                                                      ctypes.POINTER(ctypes.c_int64)]),
        "dcflow_n1_worst_per_case_workspace_bytes": (ctypes.c_int, [P, I32, ctypes.POINTER(SZ)]),
        "dcflow_n1_worst_per_case": (ctypes.c_int, [P, P, I32, ctypes.c_int, P, I32, I32, P, SZ,
                                                    P, P]),
        "dcflow_fold_stubs": (ctypes.c_int, [I32, I32, I32, P, P, P, P, P, P,
                                             ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "dcflow_fold_injections": (ctypes.c_int, [I32, P, I32, P, I32, P]),
        "dcflow_stub_flows": (ctypes.c_int, [I32, I32, P, P, P, P, I32, P]),
        "dcflow_batch_bytes": (ctypes.c_int, [P, P, I32, ctypes.POINTER(SZ)]),
        "dcflow_batch_create": (ctypes.c_int, [P, P, I32, P, SZ, P, ctypes.POINTER(P)]),
        "dcflow_batch_destroy": (None, [P]),
        "dcflow_eval_topologies": (ctypes.c_int, [P, P]),
        "dcflow_flow_bytes": (ctypes.c_int, [P, I32, ctypes.c_int, ctypes.POINTER(SZ),
                                             ctypes.POINTER(I32)]),
        "dcflow_eval_injections": (ctypes.c_int, [P, P, I32, I32, ctypes.c_int, P, SZ, P]),
        "dcflow_n1_score": (ctypes.c_int, [P, P, I32, ctypes.c_int, P, P]),
        "dcflow_batch_variant_max": (P, [P]),
        "dcflow_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "dcflow_mlp_param_count": (ctypes.c_int, []),
        "dcflow_mlp_bf16_bytes": (SZ, []),
        "dcflow_mlp_workspace_bytes": (SZ, [I32]),
        "dcflow_snapshot_flows": (ctypes.c_int, [P, P, I32, P, P, P]),
        "dcflow_n1_worst_workspace_bytes": (ctypes.c_int, [P, I32, P]),
        "dcflow_n1_worst": (ctypes.c_int, [P, P, I32, ctypes.c_int, P, I32, P, SZ, P, P]),
        "dcflow_n1_worst_noalloc": (ctypes.c_int, [P, P, I32, ctypes.c_int, P, I32, P, P]),
        "dcflow_step": (ctypes.c_int, [P, P, I32, I32, ctypes.c_int, P, SZ, P, P]),
        "dcflow_set_busbar_injections": (ctypes.c_int, [P, P, I32]),
        "dcflow_batch_set_tuning": (ctypes.c_int, [P, P]),
        "dcflow_batch_get_tuning": (ctypes.c_int, [P, P]),
        "dcflow_graph_capture": (ctypes.c_int, [P, P, I32, I32, ctypes.c_int, P, SZ, P, P]),
        "dcflow_graph_launch": (ctypes.c_int, [P, P]),
        "dcflow_snapshot_pairs": (ctypes.c_int, [P, P, I32, P, P, P]),
        "dcflow_action_features": (ctypes.c_int, [P, P, P, P, P, P, I32, P, P, P, P, P, P]),
        "dcflow_improvement_labels": (ctypes.c_int, [P, P, P, I32, P, P]),
        "dcflow_mlp_forward": (ctypes.c_int, [P, P, I32, P, P, SZ, P]),
        "dcflow_mlp_grad": (ctypes.c_int, [P, P, P, I32, P, P, P, SZ, P]),
        "dcflow_mlp_adam": (ctypes.c_int, [P, P, P, P, I32, ctypes.c_float, P]),
        "dcflow_mlp_pack_bf16": (ctypes.c_int, [P, P, P]),
        "dcflow_mlp_infer": (ctypes.c_int, [P, P, P, I32, P, P]),
        "dcflow_column_stats": (ctypes.c_int, [P, I32, I32, P, P, P]),
        "dcflow_standardize": (ctypes.c_int, [P, ctypes.c_int64, I32, P, P, P]),
        "dcflow_topk_smallest": (ctypes.c_int, [P, I32, I32, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("dcflow_plan_workspace_bytes", "dcflow_build_ptdf", "dcflow_plan_view_get",
            "dcflow_plan_destroy", "dcflow_validate_candidates", "dcflow_batch_bytes",
            "dcflow_batch_create", "dcflow_batch_destroy", "dcflow_eval_topologies",
            "dcflow_flow_bytes", "dcflow_eval_injections", "dcflow_n1_score",
            "dcflow_batch_variant_max", "dcflow_strerror", "dcflow_n1_worst_workspace_bytes",
            "dcflow_n1_worst", "dcflow_n1_worst_noalloc", "dcflow_step",
            "dcflow_set_busbar_injections",
            "dcflow_fold_stubs", "dcflow_fold_injections", "dcflow_stub_flows",
            "dcflow_n1_worst_per_case_workspace_bytes", "dcflow_n1_worst_per_case",
            "dcflow_batch_set_tuning",
            "dcflow_batch_get_tuning", "dcflow_graph_capture", "dcflow_graph_launch", "dcflow_mlp_param_count",
            "dcflow_mlp_bf16_bytes", "dcflow_mlp_workspace_bytes", "dcflow_snapshot_flows",
            "dcflow_snapshot_pairs", "dcflow_action_features", "dcflow_improvement_labels",
            "dcflow_mlp_forward", "dcflow_mlp_grad", "dcflow_mlp_adam",
            "dcflow_mlp_pack_bf16", "dcflow_mlp_infer", "dcflow_column_stats",
            "dcflow_standardize", "dcflow_topk_smallest")


def _check(rc, what, bad=None):
    if rc != 0:
        raise DcflowError(rc, what, bad)


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class _GridArgs:
    """Keeps the host arrays of a grid description alive."""

    def __init__(self, n_bus, f, t, b, mon, out, p_base, slack=0, rating=None,
                 rating_scale=1.2, rating_offset=0.1, controls=None, gens=None, multi=None):
        """controls: None or dict(pst=[branch ids], pst_scale=rad per unit,
        hvdc=[(from bus, to bus)], hvdc_scale=p.u. per unit).
        gens: None or (bus ids, lost outputs) of the generator-outage N-1 cases.
        multi: None or a list of branch-id lists, the multi-outage N-1 cases."""
        c = controls or {}
        gb, gp = ([], []) if gens is None else gens
        self.gen_bus = _arr(gb, np.int32)
        self.gen_p = _arr(gp, np.float64)
        assert len(self.gen_bus) == len(self.gen_p)
        cases = [] if multi is None else [list(c) for c in multi]
        self.multi_off = _arr(np.cumsum([0] + [len(c) for c in cases]), np.int32)
        self.multi_br = _arr([x for c in cases for x in c], np.int32)
        self.pst = _arr(c.get("pst", []), np.int32)
        hv = np.asarray(c.get("hvdc", []), np.int32).reshape(-1, 2)
        self.hv_from = _arr(hv[:, 0], np.int32)
        self.hv_to = _arr(hv[:, 1], np.int32)
        self.f = _arr(f, np.int32)
        self.t = _arr(t, np.int32)
        self.b = _arr(b, np.float64)
        self.mon = _arr(mon, np.int32)
        self.out = _arr(out, np.int32)
        self.p = _arr(p_base, np.float64)
        self.r = None if rating is None else _arr(rating, np.float64)
        self.desc = GridDesc(
            int(n_bus), len(self.f), int(slack), self.f.ctypes.data, self.t.ctypes.data,
            self.b.ctypes.data, len(self.mon), self.mon.ctypes.data, len(self.out),
            self.out.ctypes.data if len(self.out) else None, self.p.ctypes.data,
            None if self.r is None else self.r.ctypes.data, float(rating_scale),
            float(rating_offset), len(self.pst), self.pst.ctypes.data if len(self.pst) else None,
            float(c.get("pst_scale", np.pi / 180.0)), len(self.hv_from),
            self.hv_from.ctypes.data if len(self.hv_from) else None,
            self.hv_to.ctypes.data if len(self.hv_to) else None,
            float(c.get("hvdc_scale", 1.0)), len(self.gen_bus),
            self.gen_bus.ctypes.data if len(self.gen_bus) else None,
            self.gen_p.ctypes.data if len(self.gen_p) else None, len(cases),
            self.multi_off.ctypes.data if cases else None,
            self.multi_br.ctypes.data if len(self.multi_br) else None)


class _CandArgs:
    def __init__(self, off, kind, ids, mask, p_new=None):
        self.off = _arr(off, np.int32)
        self.kind = _arr(kind, np.int8)
        self.id = _arr(ids, np.int32)
        self.mask = _arr(mask, np.uint32)
        self.p_new = None if p_new is None else _arr(p_new, np.float64)
        ne = len(self.kind)
        self.desc = Cands(len(self.off) - 1, self.off.ctypes.data,
                          self.kind.ctypes.data if ne else None,
                          self.id.ctypes.data if ne else None,
                          self.mask.ctypes.data if ne else None,
                          None if self.p_new is None or ne == 0 else self.p_new.ctypes.data)


def cand_args(cands):
    """Candidate arrays from any object with off/kind/id/mask/p_new attributes."""
    return _CandArgs(cands.off, cands.kind, cands.id, cands.mask, getattr(cands, "p_new", None))


def fold_stubs(n_bus, f, t, slack=0, protect=None):
    """dcflow_fold_stubs (host): returns dict(bus_new, branch_new, up_branch, n_bus,
    n_branch, slack) of the folded grid; ``protect`` is a boolean [n_bus] or None."""
    f = _arr(f, np.int32)
    t = _arr(t, np.int32)
    pr = None if protect is None else _arr(np.asarray(protect, bool), np.uint8)
    bus_new = np.empty(int(n_bus), np.int32)
    branch_new = np.empty(len(f), np.int32)
    up = np.empty(int(n_bus), np.int32)
    nb, nl = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(_lib.dcflow_fold_stubs(int(n_bus), len(f), int(slack), f.ctypes.data, t.ctypes.data,
                                  None if pr is None else pr.ctypes.data, bus_new.ctypes.data,
                                  branch_new.ctypes.data, up.ctypes.data, ctypes.byref(nb),
                                  ctypes.byref(nl)), "dcflow_fold_stubs")
    return dict(bus_new=bus_new, branch_new=branch_new, up_branch=up, n_bus=nb.value,
                n_branch=nl.value, slack=int(bus_new[int(slack)]))


def fold_injections(fold, x):
    """dcflow_fold_injections (host): x [n_var][n_bus] -> [n_var][fold n_bus]."""
    x = _arr(np.atleast_2d(x), np.float64)
    out = np.empty((x.shape[0], fold["n_bus"]), np.float64)
    _check(_lib.dcflow_fold_injections(x.shape[1], fold["bus_new"].ctypes.data, fold["n_bus"],
                                       x.ctypes.data, x.shape[0], out.ctypes.data),
           "dcflow_fold_injections")
    return out


def stub_flows(fold, f, t, x):
    """dcflow_stub_flows (host): flows [n_var][n_branch] of the folded branches."""
    f = _arr(f, np.int32)
    t = _arr(t, np.int32)
    x = _arr(np.atleast_2d(x), np.float64)
    out = np.empty((x.shape[0], len(f)), np.float64)
    _check(_lib.dcflow_stub_flows(x.shape[1], len(f), f.ctypes.data, t.ctypes.data,
                                  fold["up_branch"].ctypes.data, x.ctypes.data, x.shape[0],
                                  out.ctypes.data), "dcflow_stub_flows")
    return out


def validate_candidates(grid_args: _GridArgs, cands):
    """Host-only validation; returns (packed_slots, padded_slots)."""
    ca = cands if isinstance(cands, _CandArgs) else cand_args(cands)
    bad = ctypes.c_int32(0)
    packed = ctypes.c_int64(0)
    padded = ctypes.c_int64(0)
    rc = _lib.dcflow_validate_candidates(ctypes.byref(grid_args.desc), ctypes.byref(ca.desc),
                                         ctypes.byref(bad), ctypes.byref(packed),
                                         ctypes.byref(padded))
    _check(rc, "dcflow_validate_candidates", bad.value if rc == -6 else None)
    return packed.value, padded.value


class Plan:
    """dcflow_build_ptdf: one-time FP64 base build on the current CUDA device."""

    def __init__(self, n_bus, f, t, b, mon, out, p_base, slack=0, rating=None,
                 rating_scale=1.2, rating_offset=0.1, device="cuda", stream=None, controls=None,
                 gens=None, multi=None):
        import torch
        self.args = _GridArgs(n_bus, f, t, b, mon, out, p_base, slack, rating, rating_scale,
                              rating_offset, controls, gens, multi)
        nbytes = ctypes.c_size_t(0)
        _check(_lib.dcflow_plan_workspace_bytes(ctypes.byref(self.args.desc), ctypes.byref(nbytes)),
               "dcflow_plan_workspace_bytes")
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(_lib.dcflow_build_ptdf(ctypes.byref(self.args.desc), ctypes.c_void_p(self.ws.data_ptr()),
                                      nbytes.value, _stream(stream), ctypes.byref(h)),
               "dcflow_build_ptdf")
        self.h = h
        self.device = device
        v = PlanView()
        _check(_lib.dcflow_plan_view_get(h, ctypes.byref(v)), "dcflow_plan_view_get")
        self.view = v

    @classmethod
    def from_workload(cls, w, rating=None, **kw):
        g = w.grid
        kw.setdefault("controls", getattr(w, "controls", None))
        kw.setdefault("gens", getattr(w, "gens", None))
        kw.setdefault("multi", getattr(w, "multi", None))
        return cls(g.n_bus, g.f, g.t, g.b, w.mon, w.out, g.p, g.slack, rating,
                   w.rating_scale, w.rating_offset, **kw)

    def _dev(self, ptr, shape, dtype):
        import torch
        n = int(np.prod(shape))
        el = torch.empty(0, dtype=dtype).element_size()
        base = self.ws.data_ptr()
        off = ptr - base
        assert off % el == 0 and 0 <= off and off + n * el <= self.ws.numel()
        return self.ws[off:off + n * el].view(dtype).view(*shape)

    def ptdf(self, controls=False):
        """PTDF [n_branch][n_bus], with controls=True [n_branch][n_inj] including the
        phase-shifter and HVDC columns."""
        import torch
        v = self.view
        return self._dev(v.ptdf, (v.n_branch, v.ld_h), torch.float64)[
            :, : (v.n_inj if controls else v.n_bus)]

    def hdo(self, gens=False):
        """Contingency columns [n_branch][n_out] (with gens=True also the generator
        columns PTDF[:, bus_g], [n_branch][n_out + n_gen_out])."""
        import torch
        v = self.view
        return self._dev(v.hdo, (v.n_branch, v.ld_o), torch.float64)[
            :, :v.n_out + (v.n_gen_out if gens else 0)]

    def f_base(self):
        import torch
        return self._dev(self.view.f_base, (self.view.n_branch,), torch.float64)

    def rating(self):
        import torch
        return self._dev(self.view.rating, (self.view.n_mon,), torch.float64)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:  # module globals may already be gone at interpreter exit
            _lib.dcflow_plan_destroy(h)
            self.h = None


class Batch:
    """dcflow_batch_create (validate, pack, upload) plus the three per-batch calls."""

    def __init__(self, plan: Plan, cands, n_var_max: int, stream=None):
        import torch
        self.plan = plan
        self.ca = cands if isinstance(cands, _CandArgs) else cand_args(cands)
        nbytes = ctypes.c_size_t(0)
        _check(_lib.dcflow_batch_bytes(plan.h, ctypes.byref(self.ca.desc), int(n_var_max),
                                       ctypes.byref(nbytes)), "dcflow_batch_bytes")
        self.buf = torch.empty(nbytes.value, dtype=torch.uint8, device=plan.device)
        h = ctypes.c_void_p()
        rc = _lib.dcflow_batch_create(plan.h, ctypes.byref(self.ca.desc), int(n_var_max),
                                      ctypes.c_void_p(self.buf.data_ptr()), nbytes.value,
                                      _stream(stream), ctypes.byref(h))
        if rc == -6:
            validate_candidates(plan.args, self.ca)   # raises with the bad index
        _check(rc, "dcflow_batch_create")
        self.h = h
        self.n_cand = len(self.ca.off) - 1
        self.n_var_max = int(n_var_max)

    def eval_topologies(self, stream=None):
        _check(_lib.dcflow_eval_topologies(self.h, _stream(stream)), "dcflow_eval_topologies")

    def flow_buffer(self, n_var, prec):
        import torch
        nbytes = ctypes.c_size_t(0)
        ld = ctypes.c_int32(0)
        _check(_lib.dcflow_flow_bytes(self.h, int(n_var), PREC[prec], ctypes.byref(nbytes),
                                      ctypes.byref(ld)), "dcflow_flow_bytes")
        dt = torch.float64 if prec == "fp64" else torch.float32
        el = 8 if prec == "fp64" else 4
        t = torch.empty(nbytes.value // el, dtype=dt, device=self.plan.device)
        return t, ld.value

    def eval_injections(self, inj, n_var, shared, prec, flows=None, stream=None):
        """inj: CUDA float64 tensor [n_cand, n_var, n_bus] or [n_var, n_bus] (shared).
        Returns the flow tensor viewed as [n_cand, n_var, ld_f]."""
        import torch
        assert inj.is_cuda and inj.dtype == torch.float64 and inj.is_contiguous()
        if flows is None:
            flows, _ = self.flow_buffer(n_var, prec)
        _check(_lib.dcflow_eval_injections(self.h, ctypes.c_void_p(inj.data_ptr()), int(n_var),
                                           int(bool(shared)), PREC[prec],
                                           ctypes.c_void_p(flows.data_ptr()),
                                           flows.numel() * flows.element_size(), _stream(stream)),
               "dcflow_eval_injections")
        self.flows = flows
        return flows

    def flows_view(self, flows, n_var):
        ld = _ld_er(self)
        return flows[: self.n_cand * n_var * ld].view(self.n_cand, n_var, ld)

    def n1_score(self, flows, n_var, prec, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(max(self.n_cand, 1) * SCORE_DTYPE.itemsize, dtype=torch.uint8,
                              device=self.plan.device)
        _check(_lib.dcflow_n1_score(self.h, ctypes.c_void_p(flows.data_ptr()), int(n_var),
                                    PREC[prec], ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "dcflow_n1_score")
        return out

    def n1_worst(self, flows, n_var, prec, scores, top_k, out=None, stream=None):
        """The top_k worst cases of every candidate's winning variant (agg_i);
        `scores` is the device output of n1_score on the same flows.  Returns a
        device uint8 tensor of n_cand x top_k CASE_DTYPE records."""
        import torch
        nb = ctypes.c_size_t(0)
        _check(_lib.dcflow_n1_worst_workspace_bytes(self.h, int(top_k), ctypes.byref(nb)),
               "dcflow_n1_worst_workspace_bytes")
        ws = torch.empty(nb.value, dtype=torch.uint8, device=self.plan.device)
        if out is None:
            out = torch.empty(max(self.n_cand, 1) * int(top_k) * CASE_DTYPE.itemsize,
                              dtype=torch.uint8, device=self.plan.device)
        _check(_lib.dcflow_n1_worst(self.h, ctypes.c_void_p(flows.data_ptr()), int(n_var),
                                    PREC[prec], ctypes.c_void_p(scores.data_ptr()), int(top_k),
                                    ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(nb.value),
                                    ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "dcflow_n1_worst")
        self._worst_ws = ws  # kept until the stream is done with it (next call or object end)
        return out

    def n1_worst_noalloc(self, flows, n_var, prec, scores, top_k, out, stream=None):
        """n1_worst through the allocation-free entry point (the library's fixed
        scratch array instead of a workspace); `out` is the caller's device
        buffer of n_cand x top_k CASE_DTYPE records."""
        _check(_lib.dcflow_n1_worst_noalloc(self.h, ctypes.c_void_p(flows.data_ptr()),
                                            int(n_var), PREC[prec],
                                            ctypes.c_void_p(scores.data_ptr()), int(top_k),
                                            ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "dcflow_n1_worst_noalloc")
        return out

    def n1_worst_per_case(self, flows, n_var, prec, scores, per_case, top_k, out=None,
                          stream=None):
        """agg_i in two levels: the top per_case loads of every case of the winning
        variant, then the top_k of their collection.  Same output as n1_worst."""
        import torch
        nb = ctypes.c_size_t(0)
        _check(_lib.dcflow_n1_worst_per_case_workspace_bytes(self.h, int(per_case),
                                                             ctypes.byref(nb)),
               "dcflow_n1_worst_per_case_workspace_bytes")
        ws = torch.empty(nb.value, dtype=torch.uint8, device=self.plan.device)
        if out is None:
            out = torch.empty(max(self.n_cand, 1) * int(top_k) * CASE_DTYPE.itemsize,
                              dtype=torch.uint8, device=self.plan.device)
        _check(_lib.dcflow_n1_worst_per_case(
            self.h, ctypes.c_void_p(flows.data_ptr()), int(n_var), PREC[prec],
            ctypes.c_void_p(scores.data_ptr()), int(per_case), int(top_k),
            ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(nb.value),
            ctypes.c_void_p(out.data_ptr()), _stream(stream)), "dcflow_n1_worst_per_case")
        self._worst_ws = ws
        return out

    @staticmethod
    def cases_to_numpy(out, n_cand, top_k):
        raw = out.cpu().numpy()[: n_cand * top_k * CASE_DTYPE.itemsize]
        return raw.view(CASE_DTYPE).reshape(n_cand, top_k)

    def set_tuning(self, scan_vc=0, scan_rchunk=0, persistent=0, scan_band=0, step_chunks=0,
                   worst_record=0, guard_tol=0.0):
        t = Tuning(int(scan_vc), int(scan_rchunk), int(persistent), int(scan_band),
                   int(step_chunks), int(worst_record), float(guard_tol))
        _check(_lib.dcflow_batch_set_tuning(self.h, ctypes.byref(t)), "dcflow_batch_set_tuning")

    def get_tuning(self):
        t = Tuning()
        _check(_lib.dcflow_batch_get_tuning(self.h, ctypes.byref(t)), "dcflow_batch_get_tuning")
        return t.as_dict()

    def capture(self, inj, n_var, shared, prec, flows, out, stream):
        """Captures the whole step (dcflow_step: eval_topologies -> eval_injections
        -> n1_score, in the tuning's step chunks) with these buffers into the
        batch's HIP graph (stream: a torch.cuda.Stream, not the null stream);
        replay() then runs it with one launch."""
        _check(_lib.dcflow_graph_capture(self.h, ctypes.c_void_p(inj.data_ptr()), int(n_var),
                                         int(bool(shared)), PREC[prec],
                                         ctypes.c_void_p(flows.data_ptr()),
                                         flows.numel() * flows.element_size(),
                                         ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "dcflow_graph_capture")

    def set_busbar_injections(self, pnew=None, n_var=0):
        """Per-variant injections on the splits' new busbars (injection topologies):
        a float64 device tensor [n_elem][n_var], or None for the candidates' fixed
        p_new.  The tensor must stay alive while evaluations use it."""
        if pnew is None:
            _check(_lib.dcflow_set_busbar_injections(self.h, None, 0), "dcflow_set_busbar_injections")
            self._pnv = None
            return
        assert pnew.dtype.is_floating_point and pnew.element_size() == 8 and pnew.is_contiguous()
        _check(_lib.dcflow_set_busbar_injections(self.h, ctypes.c_void_p(pnew.data_ptr()), int(n_var)),
               "dcflow_set_busbar_injections")
        self._pnv = pnew

    def step(self, inj, n_var, shared, prec, flows, out, stream=None):
        """The whole step (eval_topologies, eval_injections, n1_score) in one call,
        in the tuning's step chunks (see dcflow_step)."""
        _check(_lib.dcflow_step(self.h, ctypes.c_void_p(inj.data_ptr()), int(n_var),
                                int(bool(shared)), PREC[prec], ctypes.c_void_p(flows.data_ptr()),
                                flows.numel() * flows.element_size(),
                                ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "dcflow_step")
        return out

    def replay(self, stream=None):
        _check(_lib.dcflow_graph_launch(self.h, _stream(stream)), "dcflow_graph_launch")

    def variant_max(self, n_var):
        import torch
        ptr = _lib.dcflow_batch_variant_max(self.h)
        off = ptr - self.buf.data_ptr()
        n = self.n_cand * self.n_var_max
        return self.buf[off:off + 8 * n].view(torch.float64).view(self.n_cand, self.n_var_max)[:, :n_var]

    @staticmethod
    def scores_to_numpy(out, n_cand):
        raw = out.cpu().numpy()[: n_cand * SCORE_DTYPE.itemsize]
        return raw.view(SCORE_DTYPE)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:  # module globals may already be gone at interpreter exit
            _lib.dcflow_batch_destroy(h)
            self.h = None


def _ld_er(batch):
    nbytes = ctypes.c_size_t(0)
    ld = ctypes.c_int32(0)
    _check(_lib.dcflow_flow_bytes(batch.h, 1, DCFLOW_FP64, ctypes.byref(nbytes), ctypes.byref(ld)),
           "dcflow_flow_bytes")
    return ld.value


# ---- the C entry points under their own names ---------------------------------------------

def build_ptdf(n_bus, f, t, b, mon, out, p_base, slack=0, rating=None, rating_scale=1.2,
               rating_offset=0.1, device="cuda", stream=None) -> Plan:
    return Plan(n_bus, f, t, b, mon, out, p_base, slack, rating, rating_scale, rating_offset,
                device, stream)


def eval_topologies(plan: Plan, cands, n_var_max: int, stream=None) -> Batch:
    bt = Batch(plan, cands, n_var_max, stream)
    bt.eval_topologies(stream)
    return bt


def eval_injections(batch: Batch, inj, n_var, shared, prec="fp32", stream=None):
    return batch.eval_injections(inj, n_var, shared, prec, stream=stream)


def n1_score(batch: Batch, flows, n_var, prec="fp32", stream=None):
    return batch.n1_score(flows, n_var, prec, stream=stream)


def screen(plan: Plan, cands, inj, n_var, shared, prec="fp32", stream=None):
    """Whole path for one batch; returns the numpy score records."""
    import torch
    bt = eval_topologies(plan, cands, n_var, stream)
    flows = eval_injections(bt, inj, n_var, shared, prec, stream)
    out = n1_score(bt, flows, n_var, prec, stream)
    torch.cuda.synchronize()
    return Batch.scores_to_numpy(out, bt.n_cand), bt, flows
