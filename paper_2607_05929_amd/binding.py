"""ctypes binding of ``include/fmsolve.h`` (argument marshalling only).

Every step of the solver runs in the HIP library ``libfmsolve.so``; this
module only mirrors the C structures, turns ``workloads.Problem`` objects
into them and hands torch-allocated device buffers and the current HIP
stream to the library.  Importing it fails loudly when the library has not
been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmsolve.so")

FM_OK, FM_W_NOT_CONVERGED = 0, 1


class FmError(RuntimeError):
    pass


class PlanDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double), ("bc", C.c_int32 * 18),
                ("scheme", C.c_int32), ("green", C.c_int32), ("lambda0", C.c_double),
                ("mu0", C.c_double), ("prec", C.c_int32), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("aa_depth", C.c_int32), ("aa_period", C.c_int32),
                ("max_materials", C.c_int32), ("with_state", C.c_int32), ("finite_strain", C.c_int32)]


class Material(C.Structure):
    _fields_ = [("law", C.c_int32), ("pad_", C.c_int32), ("p", C.c_double * 8),
                ("quat", C.c_double * 4)]


class LoadStep(C.Structure):
    _fields_ = [("c", C.c_double * 3), ("G", C.c_double * 9), ("H", C.c_double * 27),
                ("mixed_mask", C.c_int32 * 6), ("mixed_target", C.c_double * 6),
                ("dt", C.c_double), ("traction", C.c_double * 18), ("ustar", C.c_void_p)]


class Outputs(C.Structure):
    _fields_ = [("u", C.c_void_p), ("eps", C.c_void_p), ("sig", C.c_void_p),
                ("macro_sigma", C.POINTER(C.c_double)), ("iters", C.POINTER(C.c_int32)),
                ("converged", C.POINTER(C.c_int32))]


class IterEntry(C.Structure):
    _fields_ = [("step", C.c_int32), ("iter", C.c_int32), ("err", C.c_double),
                ("aa_applied", C.c_int32), ("rs_fp64", C.c_int32), ("macro_sigma", C.c_double * 6),
                ("t_us", C.c_double)]


class IterLog(C.Structure):
    _fields_ = [("entries", C.POINTER(IterEntry)), ("capacity", C.c_int32), ("count", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("desc", PlanDesc), ("mat_id", C.POINTER(C.c_int32)), ("n_mat", C.c_int32),
                ("table", C.POINTER(Material)), ("steps", C.POINTER(LoadStep)),
                ("n_steps", C.c_int32), ("macro_sigma", C.POINTER(C.c_double)),
                ("iters", C.POINTER(C.c_int32)), ("arrival_s", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("completed", C.c_int64), ("admitted", C.c_int64), ("waiting", C.c_int64),
                ("active", C.c_int64), ("rejected", C.c_int64), ("p50_latency_s", C.c_double),
                ("p99_latency_s", C.c_double), ("mean_latency_s", C.c_double),
                ("voxel_iters", C.c_double), ("arena_in_use", C.c_size_t),
                ("arena_peak", C.c_size_t)]


EXPORTS = {
    "fm_workspace_bytes": (C.c_size_t, [C.POINTER(PlanDesc)]),
    "fm_plan_create": (C.c_int, [C.POINTER(PlanDesc), C.c_void_p, C.c_size_t, C.c_void_p,
                                 C.POINTER(C.c_void_p)]),
    "fm_set_material": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(Material)]),
    "fm_solve": (C.c_int, [C.c_void_p, C.POINTER(LoadStep), C.c_int32, C.POINTER(Outputs),
                           C.POINTER(IterLog)]),
    "fm_batch_workspace_bytes": (C.c_size_t, [C.POINTER(C.c_void_p), C.c_int32]),
    "fm_batch_solve": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.POINTER(LoadStep)),
                                 C.POINTER(C.c_int32), C.POINTER(Outputs), C.POINTER(IterLog),
                                 C.POINTER(C.c_int32), C.c_void_p, C.c_size_t]),
    "fm_apply_green": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fm_residual": (C.c_int, [C.c_void_p, C.POINTER(LoadStep), C.c_void_p, C.c_void_p,
                              C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "fm_profile_iterations": (C.c_int, [C.c_void_p, C.POINTER(LoadStep), C.c_int32,
                                        C.POINTER(C.c_double)]),
    "fm_plan_total_iterations": (C.c_int64, [C.c_void_p]),
    "fm_plan_destroy": (None, [C.c_void_p]),
    "fm_server_create": (C.c_int, [C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p,
                                   C.POINTER(C.c_void_p)]),
    "fm_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.c_double,
                                   C.POINTER(C.c_uint64)]),
    "fm_server_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_double]),
    "fm_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32),
                                 C.POINTER(C.c_double)]),
    "fm_server_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "fm_server_destroy": (None, [C.c_void_p]),
    "fm_last_error": (C.c_char_p, []),
    "fm_solve_static": (C.c_int, [C.POINTER(PlanDesc), C.c_void_p, C.c_int32, C.POINTER(Material),
                                  C.POINTER(LoadStep), C.c_int32, C.POINTER(Outputs), C.POINTER(IterLog),
                                  C.c_void_p]),
    "fm_set_graph_launch": (C.c_int, [C.c_int]),
    "fm_autotune": (C.c_int, [C.c_void_p, C.POINTER(LoadStep), C.c_int32, C.POINTER(C.c_int32),
                              C.POINTER(C.c_double)]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FmError(f"HIP library not built: {LIB_PATH} missing (run __graft_entry__.build())")
        # torch ships its own HIP runtime; load it first so the library binds
        # to the same runtime (one HIP/HSA runtime per process, matched by soname)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc, what=""):
    if rc < 0:
        msg = lib().fm_last_error().decode()
        raise FmError(f"{what} failed ({rc}): {msg}")
    return rc


# --------------------------------------------------------------------------
# Marshalling of workloads.Problem
# --------------------------------------------------------------------------
def plan_desc(prob, prec=None) -> PlanDesc:
    d = PlanDesc()
    for i in range(3):
        d.n[i] = int(prob.n[i])
    d.h = float(prob.h)
    bc = np.asarray(prob.bc, dtype=np.int32).reshape(-1)
    for i in range(18):
        d.bc[i] = int(bc[i])
    d.scheme = int(prob.scheme)
    d.green = int(prob.green)
    d.lambda0 = float(prob.lambda0)
    d.mu0 = float(prob.mu0)
    d.prec = int(prob.prec if prec is None else prec)
    d.tol = float(prob.tol)
    d.max_iter = int(prob.max_iter)
    d.aa_depth = int(prob.aa_depth)
    d.aa_period = int(prob.aa_period)
    d.max_materials = max(1, len(prob.materials))
    d.with_state = int(any(m["law"] in (2, 3) for m in prob.materials))
    d.finite_strain = int(getattr(prob, "finite_strain", 0))
    return d


def material_table(prob):
    arr = (Material * len(prob.materials))()
    for k, m in enumerate(prob.materials):
        e = arr[k]
        e.law = int(m["law"])
        if m["law"] == 0:
            vals = [m["lam"], m["mu"]]
        elif m["law"] == 1:
            vals = [m["C11"], m["C12"], m["C44"]]
        elif m["law"] == 2:
            vals = [m["lam"], m["mu"], m["sy0"], m["H"]]
        elif m["law"] == 4:
            vals = [m["lam"], m["mu"]]
        elif m["law"] == 5:
            vals = [m["mu"], m["K"]]
        else:
            vals = [m["C11"], m["C12"], m["C44"], m["gdot0"], m["n"], m["tau0"], m["taus"],
                    m["theta0"]]
        for i, v in enumerate(vals):
            e.p[i] = float(v)
        q = m.get("quat", [1.0, 0.0, 0.0, 0.0])
        for i in range(4):
            e.quat[i] = float(q[i])
    return arr


def load_steps(steps):
    arr = (LoadStep * len(steps))()
    keep = []
    for k, s in enumerate(steps):
        e = arr[k]
        for i in range(3):
            e.c[i] = float(s.c[i])
        G = np.asarray(s.G, dtype=np.float64).reshape(-1)
        H = np.asarray(s.H, dtype=np.float64).reshape(-1)
        for i in range(9):
            e.G[i] = G[i]
        for i in range(27):
            e.H[i] = H[i]
        for i in range(6):
            e.mixed_mask[i] = int(s.mixed_mask[i])
            e.mixed_target[i] = float(s.mixed_target[i])
        e.dt = float(s.dt)
        T = np.asarray(getattr(s, "traction", np.zeros((3, 2, 3))), dtype=np.float64).reshape(-1)
        for i in range(18):
            e.traction[i] = T[i]
        nod = getattr(s, "ustar_nodal", None)
        if nod is not None:
            # (3, N1, N2, N3) -> the library's node layout (3, N3, N2, N1), on the device;
            # the array keeps the tensor alive as long as the steps are in use
            torch = _torch()
            t = torch.from_numpy(np.ascontiguousarray(np.asarray(nod, dtype=np.float64).transpose(0, 3, 2, 1)))
            t = t.to("cuda")
            keep.append(t)
            e.ustar = t.data_ptr()
    arr._keep = keep
    return arr


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise FmError("no HIP device visible to torch")
    return torch


def _stream_ptr(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """One solve: workspace and buffers are torch tensors on the current device."""

    def __init__(self, prob, prec=None):
        torch = _torch()
        self.torch = torch
        self.prob = prob
        self.desc = plan_desc(prob, prec)
        L = lib()
        self.ws_bytes = int(L.fm_workspace_bytes(C.byref(self.desc)))
        if self.ws_bytes == 0:
            raise FmError("invalid plan descriptor: " + L.fm_last_error().decode())
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.handle = C.c_void_p()
        check(L.fm_plan_create(C.byref(self.desc), C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                               _stream_ptr(torch), C.byref(self.handle)), "fm_plan_create")
        self.n = tuple(int(v) for v in prob.n)
        self.nppv = 2 if prob.scheme == 1 else 1
        self.set_material(prob.mat_id, prob.materials)

    def set_material(self, mat_id, materials):
        torch = self.torch
        self._ids = torch.as_tensor(np.ascontiguousarray(mat_id, dtype=np.int32).reshape(-1),
                                    device="cuda")
        self._tab = material_table(self.prob)
        check(lib().fm_set_material(self.handle, C.c_void_p(self._ids.data_ptr()), len(materials),
                                    self._tab), "fm_set_material")
        torch.cuda.current_stream().synchronize()

    def output_buffers(self):
        torch = self.torch
        n1, n2, n3 = self.n
        nn = (n1 + 1) * (n2 + 1) * (n3 + 1)
        nv = n1 * n2 * n3
        return {"u": torch.empty(3 * nn, dtype=torch.float64, device="cuda"),
                "eps": torch.empty(6 * self.nppv * nv, dtype=torch.float64, device="cuda"),
                "sig": torch.empty(6 * self.nppv * nv, dtype=torch.float64, device="cuda")}

    def solve(self, steps=None, fields=True, log_capacity=0):
        torch = self.torch
        steps = self.prob.steps if steps is None else steps
        st = load_steps(steps)
        ns = len(steps)
        macro = np.zeros((ns, 6))
        iters = np.zeros(ns, dtype=np.int32)
        conv = np.zeros(ns, dtype=np.int32)
        out = Outputs()
        bufs = self.output_buffers() if fields else None
        if bufs is not None:
            out.u = bufs["u"].data_ptr(); out.eps = bufs["eps"].data_ptr(); out.sig = bufs["sig"].data_ptr()
        out.macro_sigma = macro.ctypes.data_as(C.POINTER(C.c_double))
        out.iters = iters.ctypes.data_as(C.POINTER(C.c_int32))
        out.converged = conv.ctypes.data_as(C.POINTER(C.c_int32))
        log = None
        entries = None
        if log_capacity:
            entries = (IterEntry * log_capacity)()
            log = IterLog(entries, log_capacity, 0)
        rc = check(lib().fm_solve(self.handle, st, ns, C.byref(out), C.byref(log) if log else None),
                   "fm_solve")
        torch.cuda.current_stream().synchronize()
        res = {"rc": rc, "macro_sigma": macro, "iters": iters.tolist(),
               "converged": [bool(v) for v in conv]}
        if bufs is not None:
            n1, n2, n3 = self.n
            res["u"] = bufs["u"].cpu().numpy().reshape(3, n3 + 1, n2 + 1, n1 + 1)
            res["eps"] = bufs["eps"].cpu().numpy().reshape(6, self.nppv, n3, n2, n1)
            res["sig"] = bufs["sig"].cpu().numpy().reshape(6, self.nppv, n3, n2, n1)
        if log is not None:
            res["log"] = [{"step": entries[i].step, "iter": entries[i].iter, "err": entries[i].err,
                           "aa": bool(entries[i].aa_applied), "rs_fp64": bool(entries[i].rs_fp64),
                           "macro_sigma": list(entries[i].macro_sigma), "t_us": entries[i].t_us}
                          for i in range(log.count)]
        return res

    def apply_green(self, x):
        """x: (3, n3+1, n2+1, n1+1) node field -> IDT(DT(x) / den)."""
        torch = self.torch
        xd = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64).reshape(-1), device="cuda")
        wd = torch.empty_like(xd)
        check(lib().fm_apply_green(self.handle, C.c_void_p(xd.data_ptr()), C.c_void_p(wd.data_ptr())),
              "fm_apply_green")
        n1, n2, n3 = self.n
        return wd.cpu().numpy().reshape(3, n3 + 1, n2 + 1, n1 + 1)

    def residual(self, uf, step):
        """D = div_d sigma at the nodes for fluctuation uf and load step ``step``."""
        torch = self.torch
        ud = torch.as_tensor(np.ascontiguousarray(uf, dtype=np.float64).reshape(-1), device="cuda")
        Dd = torch.empty_like(ud)
        err = C.c_double()
        macro = (C.c_double * 6)()
        st = load_steps([step])
        check(lib().fm_residual(self.handle, st, C.c_void_p(ud.data_ptr()), C.c_void_p(Dd.data_ptr()),
                                C.byref(err), macro), "fm_residual")
        n1, n2, n3 = self.n
        return Dd.cpu().numpy().reshape(3, n3 + 1, n2 + 1, n1 + 1), err.value, np.array(macro[:])

    KERNELS = ("stress_div", "control", "gram", "alpha", "x_fwd", "y_fwd", "z_green",
               "y_inv", "x_inv_update")

    def profile(self, step=None, n_iter=10):
        """Mean per-kernel duration (ms) of the iteration, from HIP events on the plan's stream."""
        step = self.prob.steps[0] if step is None else step
        ms = (C.c_double * 9)()
        check(lib().fm_profile_iterations(self.handle, load_steps([step]), n_iter, ms),
              "fm_profile_iterations")
        return dict(zip(self.KERNELS, list(ms)))

    def autotune(self, step=None, n_iter=4):
        """Pick the fastest transform kernel per axis pass (fm_autotune), then
        reset the displacement.  Returns the choices and the timing table."""
        step = self.prob.steps[0] if step is None else step
        choice = (C.c_int32 * 5)()
        ms = (C.c_double * 20)()
        check(lib().fm_autotune(self.handle, load_steps([step]), n_iter, choice, ms), "fm_autotune")
        self.reset()
        return {"choice": list(choice), "ms": np.array(ms[:]).reshape(4, 5)}

    def reset(self, sync=True):
        """Zero the displacement and internal variables (same device-resident microstructure)."""
        check(lib().fm_set_material(self.handle, C.c_void_p(self._ids.data_ptr()),
                                    len(self.prob.materials), self._tab), "fm_set_material")
        if sync:
            self.torch.cuda.current_stream().synchronize()

    def total_iterations(self):
        return int(lib().fm_plan_total_iterations(self.handle))

    def close(self):
        if self.handle:
            lib().fm_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_static(prob, prec=None):
    """fm_solve_static: one solve on the library's static device scratch (the
    library allocates nothing); outputs as Plan.solve."""
    torch = _torch()
    d = plan_desc(prob, prec)
    ids = torch.as_tensor(np.ascontiguousarray(prob.mat_id, dtype=np.int32).reshape(-1), device="cuda")
    tab = material_table(prob)
    st = load_steps(prob.steps)
    ns = len(prob.steps)
    n1, n2, n3 = (int(v) for v in prob.n)
    nppv = 2 if prob.scheme == 1 else 1
    nn = (n1 + 1) * (n2 + 1) * (n3 + 1)
    nv = n1 * n2 * n3
    bufs = {"u": torch.empty(3 * nn, dtype=torch.float64, device="cuda"),
            "eps": torch.empty(6 * nppv * nv, dtype=torch.float64, device="cuda"),
            "sig": torch.empty(6 * nppv * nv, dtype=torch.float64, device="cuda")}
    macro = np.zeros((ns, 6))
    iters = np.zeros(ns, dtype=np.int32)
    conv = np.zeros(ns, dtype=np.int32)
    out = Outputs()
    out.u = bufs["u"].data_ptr(); out.eps = bufs["eps"].data_ptr(); out.sig = bufs["sig"].data_ptr()
    out.macro_sigma = macro.ctypes.data_as(C.POINTER(C.c_double))
    out.iters = iters.ctypes.data_as(C.POINTER(C.c_int32))
    out.converged = conv.ctypes.data_as(C.POINTER(C.c_int32))
    rc = check(lib().fm_solve_static(C.byref(d), C.c_void_p(ids.data_ptr()), len(prob.materials), tab, st, ns,
                                     C.byref(out), None, _stream_ptr(torch)), "fm_solve_static")
    torch.cuda.current_stream().synchronize()
    return {"rc": rc, "macro_sigma": macro, "iters": iters.tolist(), "converged": [bool(v) for v in conv],
            "u": bufs["u"].cpu().numpy().reshape(3, n3 + 1, n2 + 1, n1 + 1),
            "eps": bufs["eps"].cpu().numpy().reshape(6, nppv, n3, n2, n1),
            "sig": bufs["sig"].cpu().numpy().reshape(6, nppv, n3, n2, n1)}


def set_graph_launch(enable: bool):
    """Process-wide launch mode of the iteration chunks: captured HIP graphs
    (default) or direct kernel launches."""
    check(lib().fm_set_graph_launch(1 if enable else 0), "fm_set_graph_launch")


def solve(prob, prec=None, fields=True, log_capacity=0):
    p = Plan(prob, prec)
    try:
        return p.solve(fields=fields, log_capacity=log_capacity)
    finally:
        p.close()


def batch_solve(problems, prec=None, fields=False, plans=None):
    """Solve independent problems together (fm_batch_solve).  `plans`:
    already created plans of the problems (kept open), else created here."""
    torch = _torch()
    own = plans is None
    if own:
        plans = []
        try:
            for p in problems:
                plans.append(Plan(p, prec))
            return batch_solve(problems, prec, fields, plans)
        finally:
            for pl in plans:
                pl.close()
    n = len(plans)
    handles = (C.c_void_p * n)(*[p.handle.value for p in plans])
    steps = [load_steps(p.steps) for p in problems]
    step_ptrs = (C.POINTER(LoadStep) * n)(*[C.cast(s, C.POINTER(LoadStep)) for s in steps])
    nsteps = (C.c_int32 * n)(*[len(p.steps) for p in problems])
    outs = (Outputs * n)()
    macros = [np.zeros((len(p.steps), 6)) for p in problems]
    iters = [np.zeros(len(p.steps), dtype=np.int32) for p in problems]
    bufs = []
    for i, pl in enumerate(plans):
        outs[i].macro_sigma = macros[i].ctypes.data_as(C.POINTER(C.c_double))
        outs[i].iters = iters[i].ctypes.data_as(C.POINTER(C.c_int32))
        if fields:
            b = pl.output_buffers()
            bufs.append(b)
            outs[i].u = b["u"].data_ptr(); outs[i].eps = b["eps"].data_ptr(); outs[i].sig = b["sig"].data_ptr()
    status = (C.c_int32 * n)()
    wsb = int(lib().fm_batch_workspace_bytes(handles, n))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    check(lib().fm_batch_solve(handles, n, step_ptrs, nsteps, outs, None, status,
                               C.c_void_p(ws.data_ptr()), wsb), "fm_batch_solve")
    torch.cuda.current_stream().synchronize()
    res = []
    for i, pl in enumerate(plans):
        r = {"rc": int(status[i]), "macro_sigma": macros[i], "iters": iters[i].tolist()}
        if fields:
            n1, n2, n3 = pl.n
            r["sig"] = bufs[i]["sig"].cpu().numpy().reshape(6, pl.nppv, n3, n2, n1)
            r["eps"] = bufs[i]["eps"].cpu().numpy().reshape(6, pl.nppv, n3, n2, n1)
        res.append(r)
    return res


class Server:
    """Continuous-batching request loop (fm_server_*) over one torch-owned arena."""

    def __init__(self, arena_bytes, max_active=64):
        torch = _torch()
        self.torch = torch
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self.handle = C.c_void_p()
        check(lib().fm_server_create(C.c_void_p(self.arena.data_ptr()), int(arena_bytes),
                                     int(max_active), _stream_ptr(torch), C.byref(self.handle)),
              "fm_server_create")
        self.keep = {}

    def submit(self, prob, arrival_s, now_s=0.0, prec=None):
        req = Request()
        req.desc = plan_desc(prob, prec)
        ids = np.ascontiguousarray(prob.mat_id, dtype=np.int32).reshape(-1)
        tab = material_table(prob)
        st = load_steps(prob.steps)
        macro = np.zeros((len(prob.steps), 6))
        iters = np.zeros(len(prob.steps), dtype=np.int32)
        req.mat_id = ids.ctypes.data_as(C.POINTER(C.c_int32))
        req.n_mat = len(prob.materials)
        req.table = tab
        req.steps = st
        req.n_steps = len(prob.steps)
        req.macro_sigma = macro.ctypes.data_as(C.POINTER(C.c_double))
        req.iters = iters.ctypes.data_as(C.POINTER(C.c_int32))
        req.arrival_s = float(arrival_s)
        t = C.c_uint64()
        check(lib().fm_server_submit(self.handle, C.byref(req), float(now_s), C.byref(t)),
              "fm_server_submit")
        # the library copies the request's inputs (a nodal u* stays on the
        # device: its tensors are kept until the result is released); it
        # writes its results into these two host arrays when the solve completes
        self.keep[t.value] = (macro, iters, st._keep)
        return t.value

    def step(self, iters, now_s):
        check(lib().fm_server_step(self.handle, int(iters), float(now_s)), "fm_server_step")

    def poll(self, ticket):
        st = C.c_int32()
        lat = C.c_double()
        check(lib().fm_server_poll(self.handle, C.c_uint64(ticket), C.byref(st), C.byref(lat)),
              "fm_server_poll")
        return int(st.value), float(lat.value)

    def result(self, ticket):
        macro, iters = self.keep[ticket][:2]
        return {"macro_sigma": macro, "iters": iters.tolist()}

    def release(self, ticket):
        """Drop the host result buffers of a completed request."""
        return self.keep.pop(ticket)

    def stats(self):
        s = Stats()
        check(lib().fm_server_stats(self.handle, C.byref(s)), "fm_server_stats")
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def close(self):
        if self.handle:
            lib().fm_server_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
