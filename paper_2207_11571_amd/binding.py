"""ctypes binding of libdgnn.so (include/dgnn.h).

Argument marshalling only: every step of the DG / network / serving path runs
in the HIP library.  PyTorch supplies device memory and the current stream.
The functions keep the C names; the small classes own the opaque handles and
the workspace tensors the calls need.
"""
import ctypes
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgnn.so")

DG_OK, DG_EINVAL, DG_ENOSPC, DG_EHIP, DG_EAGAIN, DG_ENOENT, DG_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
SOLVE_QUEUED, SOLVE_RUNNING, SOLVE_DONE, SOLVE_FAILED = 0, 1, 2, 3

_lib = None


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dgnn error {code}: {msg}")
        self.code = code


class dg_params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("P", ctypes.c_int32), ("viscous", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("L", ctypes.c_double), ("Re", ctypes.c_double),
                ("Mach", ctypes.c_double), ("gamma", ctypes.c_double), ("Pr", ctypes.c_double),
                ("Cs", ctypes.c_double), ("Pr_t", ctypes.c_double), ("p_ref", ctypes.c_double)]


class solve_request(ctypes.Structure):
    _fields_ = [("Re", ctypes.c_double), ("t_end", ctypes.c_double), ("Mach", ctypes.c_double),
                ("Cs", ctypes.c_double), ("P", ctypes.c_int32), ("N", ctypes.c_int32),
                ("use_nn", ctypes.c_int32), ("ke_every", ctypes.c_int32), ("model", ctypes.c_void_p),
                ("ke_host", ctypes.POINTER(ctypes.c_double)), ("ke_capacity", ctypes.c_int32),
                ("nn_after_step", ctypes.c_int32), ("q_out_host", ctypes.POINTER(ctypes.c_double))]


class solve_status(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("error", ctypes.c_int32), ("steps", ctypes.c_int64),
                ("n_steps", ctypes.c_int64), ("ke_count", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("t", ctypes.c_double), ("dt", ctypes.c_double), ("latency_s", ctypes.c_double),
                ("queue_s", ctypes.c_double), ("dof_updates", ctypes.c_int64), ("fallback_step", ctypes.c_int64)]


_vp, _sz, _i32, _i64, _d, _f = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float

# name -> (restype, argtypes); the full exported surface of include/dgnn.h
SIGNATURES = {
    "dg_last_error": (ctypes.c_int, [ctypes.c_char_p, _sz]),
    "dg_init_mesh": (ctypes.c_int, [ctypes.POINTER(dg_params), ctypes.POINTER(_vp)]),
    "dg_mesh_query": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_sz)]),
    "dg_free_mesh": (None, [_vp]),
    "dg_init_tgv": (ctypes.c_int, [_vp, _vp, _vp]),
    "dg_residual": (ctypes.c_int, [_vp, _vp, _vp, _vp, _sz, _vp]),
    "dg_rk_step": (ctypes.c_int, [_vp, _vp, _vp, _d, _i32, _vp, _vp, _sz, _vp]),
    "dg_rk_step_post": (ctypes.c_int, [_vp, _vp, _vp, _d, _i32, _vp, _vp, _sz, _vp]),
    "dg_rk_step_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _d, _i32, _vp, _vp]),
    "dg_profile_steps": (ctypes.c_int, [_vp, _vp, _vp, _d, _i32, _vp, _vp, _sz, _vp, ctypes.POINTER(_d)]),
    "dg_diagnostics": (ctypes.c_int, [_vp, _vp, _vp, _vp, _sz, _vp]),
    "dg_stable_dt": (ctypes.c_int, [_vp, _vp, _d, ctypes.POINTER(_d), _vp, _sz, _vp]),
    "dg_error_inf": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "dg_project": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "dg_forcing_target_ws": (_sz, [_vp, _vp]),
    "dg_forcing_target": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "dg_increment_target_ws": (_sz, [_vp, _vp]),
    "dg_increment_target": (ctypes.c_int, [_vp, _vp, _vp, _vp, _d, _i32, _vp, _vp, _vp, _sz, _vp]),
    "nn_query": (ctypes.c_int, [ctypes.POINTER(_i32), _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "nn_init": (ctypes.c_int, [ctypes.POINTER(_i32), _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                               ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_uint8), _vp, ctypes.POINTER(_vp)]),
    "nn_init_io": (ctypes.c_int, [ctypes.POINTER(_i32), _i32, _i32, ctypes.POINTER(ctypes.c_uint8),
                                  ctypes.POINTER(ctypes.c_uint8), _vp, _vp, _vp, _vp, _vp,
                                  ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_uint8), _vp, ctypes.POINTER(_vp)]),
    "nn_refresh": (ctypes.c_int, [_vp, _vp]),
    "nn_set_column_norm": (ctypes.c_int, [_vp, _vp, _i32]),
    "nn_column_stats_ws": (_sz, [_i64, _i32]),
    "nn_column_stats": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _vp, _sz, _vp]),
    "nn_set_norm": (ctypes.c_int, [_vp, ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_uint8)]),
    "nn_free": (None, [_vp]),
    "nn_forcing": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "nn_train_ws": (_sz, [_vp, _i32]),
    "nn_train_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _f, _vp, _vp, _sz, _vp]),
    "nn_stats_ws": (_sz, [_i64]),
    "nn_data_stats": (ctypes.c_int, [_vp, _vp, _i64, _i32, ctypes.POINTER(_d), _vp, _sz, _vp]),
    "solve_footprint": (_sz, [_i32, _i32, _i32]),
    "solve_server_create": (ctypes.c_int, [_vp, _sz, _i32, ctypes.POINTER(_vp)]),
    "solve_submit": (ctypes.c_int, [_vp, ctypes.POINTER(solve_request), ctypes.POINTER(ctypes.c_uint64)]),
    "solve_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(solve_status)]),
    "solve_server_drain": (ctypes.c_int, [_vp]),
    "solve_inject_nan": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "solve_server_stats": (ctypes.c_int, [_vp, ctypes.POINTER(_d), ctypes.POINTER(_i64)]),
    "solve_server_free": (None, [_vp]),
}


def lib():
    """Load libdgnn.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2207_11571_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    buf = ctypes.create_string_buffer(512)
    lib().dg_last_error(buf, 512)
    return buf.value.decode()


def check(rc, allow=()):
    if rc != DG_OK and rc not in allow:
        raise DGError(rc, last_error())
    return rc


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def make_params(N, P, Re, Mach=0.1, gamma=1.4, Pr=0.72, Cs=0.0, Pr_t=0.6, L=2.0 * math.pi, viscous=True, p_ref=None):
    p = dg_params()
    p.N, p.P, p.viscous = N, P, 1 if viscous else 0
    p.L, p.Re, p.Mach, p.gamma, p.Pr, p.Cs, p.Pr_t = L, Re, Mach, gamma, Pr, Cs, Pr_t
    p.p_ref = 1.0 / (gamma * Mach * Mach) if p_ref is None else p_ref
    return p


class Mesh:
    """dg_mesh handle plus the device workspace its calls use."""

    def __init__(self, N, P, Re, device="cuda", **kw):
        self.params = make_params(N, P, Re, **kw)
        self.N, self.P = N, P
        self.E, self.n_p = N ** 3, (P + 1) ** 3
        h = ctypes.c_void_p()
        check(lib().dg_init_mesh(ctypes.byref(self.params), ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int64()
        ws = ctypes.c_size_t()
        check(lib().dg_mesh_query(h, ctypes.byref(n), ctypes.byref(ws)))
        self.n_nodes, self.ws_bytes = n.value, ws.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.diag = torch.zeros(8, dtype=torch.float64, device=device)

    def field(self, fill=None):
        t = torch.empty((5, self.E, self.n_p), dtype=torch.float64, device=self.ws.device)
        if fill is not None:
            t.fill_(fill)
        return t

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dg_free_mesh(self.handle)
            self.handle = None


def dg_init_tgv(mesh, q, stream=None):
    check(lib().dg_init_tgv(mesh.handle, _ptr(q, torch.float64, "q"), _stream(stream)))


def dg_residual(mesh, q, dqdt, stream=None):
    check(lib().dg_residual(mesh.handle, _ptr(q, torch.float64, "q"), _ptr(dqdt, torch.float64, "dqdt"),
                            _ptr(mesh.ws), mesh.ws_bytes, _stream(stream)))


def dg_rk_step(mesh, q, k, dt, n_steps, model=None, stream=None):
    check(lib().dg_rk_step(mesh.handle, _ptr(q, torch.float64, "q"), _ptr(k, torch.float64, "k"), float(dt),
                           int(n_steps), model.handle if model is not None else None, _ptr(mesh.ws), mesh.ws_bytes,
                           _stream(stream)))


def dg_rk_step_post(mesh, q, k, dt, n_steps, model=None, stream=None):
    check(lib().dg_rk_step_post(mesh.handle, _ptr(q, torch.float64, "q"), _ptr(k, torch.float64, "k"), float(dt),
                                int(n_steps), model.handle if model is not None else None, _ptr(mesh.ws),
                                mesh.ws_bytes, _stream(stream)))


def dg_rk_step_noalloc(mesh, q, k, dt, n_steps, model=None, stream=None):
    """dg_rk_step on the library's per-GPU scratch (no workspace argument)."""
    check(lib().dg_rk_step_noalloc(mesh.handle, _ptr(q, torch.float64, "q"), _ptr(k, torch.float64, "k"),
                                   float(dt), int(n_steps), model.handle if model is not None else None,
                                   _stream(stream)))


def dg_profile_steps(mesh, q, k, dt, n_steps, model=None, stream=None):
    out = (ctypes.c_double * 4)()
    check(lib().dg_profile_steps(mesh.handle, _ptr(q, torch.float64, "q"), _ptr(k, torch.float64, "k"), float(dt),
                                 int(n_steps), model.handle if model is not None else None, _ptr(mesh.ws),
                                 mesh.ws_bytes, _stream(stream), out))
    return {"traces": out[0], "grad": out[1], "net": out[2], "resid": out[3]}


def dg_diagnostics(mesh, q, out=None, stream=None):
    out = mesh.diag if out is None else out
    check(lib().dg_diagnostics(mesh.handle, _ptr(q, torch.float64, "q"), _ptr(out, torch.float64, "out"),
                               _ptr(mesh.ws), mesh.ws_bytes, _stream(stream)))
    return out


def dg_stable_dt(mesh, q, cfl=0.4, stream=None):
    dt = ctypes.c_double()
    check(lib().dg_stable_dt(mesh.handle, _ptr(q, torch.float64, "q"), float(cfl), ctypes.byref(dt), _ptr(mesh.ws),
                             mesh.ws_bytes, _stream(stream)))
    return dt.value


def dg_error_inf(mesh, q, q_ref, out, stream=None):
    check(lib().dg_error_inf(mesh.handle, _ptr(q, torch.float64, "q"), _ptr(q_ref, torch.float64, "q_ref"),
                             _ptr(out, torch.float64, "out"), _ptr(mesh.ws), mesh.ws_bytes, _stream(stream)))
    return out


def dg_project(src, dst, f_src, f_dst, stream=None):
    check(lib().dg_project(src.handle, dst.handle, _ptr(f_src, torch.float64, "f_src"),
                           _ptr(f_dst, torch.float64, "f_dst"), _stream(stream)))


def dg_forcing_target(hi, lo, q_hi, x_out, y_out, ws=None, stream=None):
    need = lib().dg_forcing_target_ws(hi.handle, lo.handle)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=q_hi.device)
    check(lib().dg_forcing_target(hi.handle, lo.handle, _ptr(q_hi, torch.float64, "q_hi"),
                                  _ptr(x_out, torch.float32, "x_out"), _ptr(y_out, torch.float32, "y_out"),
                                  _ptr(ws), ws.numel(), _stream(stream)))
    return ws


def dg_increment_target(hi, lo, q_hi, k_hi, dt_lo, m_sub, x_out, y_out, ws=None, stream=None):
    need = lib().dg_increment_target_ws(hi.handle, lo.handle)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=q_hi.device)
    check(lib().dg_increment_target(hi.handle, lo.handle, _ptr(q_hi, torch.float64, "q_hi"),
                                    _ptr(k_hi, torch.float64, "k_hi"), float(dt_lo), int(m_sub),
                                    _ptr(x_out, torch.float32, "x_out"), _ptr(y_out, torch.float32, "y_out"),
                                    _ptr(ws), ws.numel(), _stream(stream)))
    return ws


def nn_query(dims):
    arr = (ctypes.c_int32 * len(dims))(*dims)
    n_params, n_bf16 = ctypes.c_int64(), ctypes.c_int64()
    check(lib().nn_query(arr, len(dims) - 1, ctypes.byref(n_params), ctypes.byref(n_bf16)))
    return n_params.value, n_bf16.value


def pack_params(layers):
    """[(W[out][in], b[out]), ...] -> flat float32 list in the library's order."""
    import numpy as np
    return np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()])
                           for W, b in layers])


def unpack_params(flat, dims):
    import numpy as np
    out, off = [], 0
    for a, b in zip(dims[:-1], dims[1:]):
        W = np.asarray(flat[off:off + a * b]).reshape(b, a)
        off += a * b
        bias = np.asarray(flat[off:off + b])
        off += b
        out.append((W, bias))
    return out


class Model:
    """nn_model handle plus its device buffers (float32 master, bf16 copies,
    gradient and Adam moments)."""

    def __init__(self, dims, flat_params, norm, mask=(1, 1, 1, 1, 1), activation="tanh", train=True, device="cuda",
                 stream=None, in_vars=None, out_vars=None):
        """in_vars / out_vars: the variables (indices 0..4) the network reads and
        forces; None = all five."""
        self.dims = list(dims)
        n_params, n_bf16 = nn_query(self.dims)
        self.params = torch.as_tensor(flat_params, dtype=torch.float32).to(device).contiguous()
        if self.params.numel() != n_params:
            raise ValueError(f"expected {n_params} parameters, got {self.params.numel()}")
        self.wbf = torch.zeros(n_bf16, dtype=torch.int16, device=device)
        self.grad = torch.zeros(n_params, dtype=torch.float32, device=device) if train else None
        self.m = torch.zeros(n_params, dtype=torch.float32, device=device) if train else None
        self.v = torch.zeros(n_params, dtype=torch.float32, device=device) if train else None
        arr = (ctypes.c_int32 * len(dims))(*dims)
        nrm = (ctypes.c_double * 20)(*[float(x) for x in norm])
        msk = (ctypes.c_uint8 * 5)(*[1 if x else 0 for x in mask])
        h = ctypes.c_void_p()
        def sel(vs):
            return None if vs is None else (ctypes.c_uint8 * 5)(*[1 if v in vs else 0 for v in range(5)])

        self.in_vars = tuple(range(5)) if in_vars is None else tuple(in_vars)
        self.out_vars = tuple(range(5)) if out_vars is None else tuple(out_vars)
        check(lib().nn_init_io(arr, len(dims) - 1, 0 if activation == "tanh" else 1, sel(in_vars), sel(out_vars),
                               _ptr(self.params), _ptr(self.wbf), _ptr(self.grad), _ptr(self.m), _ptr(self.v), nrm,
                               msk, _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.train_ws = None

    def set_norm(self, norm, mask=None):
        nrm = (ctypes.c_double * 20)(*[float(x) for x in norm])
        msk = (ctypes.c_uint8 * 5)(*[1 if x else 0 for x in mask]) if mask is not None else None
        check(lib().nn_set_norm(self.handle, nrm, msk))

    def set_column_norm(self, col, n_p):
        """Per-node normalisation: col is a device float64 tensor [4, 5 n_p]
        (mu_in, sigma_in, mu_out, sigma_out per row column), kept alive here;
        None returns to the per-variable maps."""
        if col is None:
            self.col_norm = None
            check(lib().nn_set_column_norm(self.handle, None, 0))
            return
        self.col_norm = col.contiguous()
        check(lib().nn_set_column_norm(self.handle, _ptr(self.col_norm, torch.float64, "col"), n_p))

    def refresh(self, stream=None):
        check(lib().nn_refresh(self.handle, _stream(stream)))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.nn_free(self.handle)
            self.handle = None


def nn_forcing(model, mesh, q, dqdt, stream=None):
    check(lib().nn_forcing(model.handle, mesh.handle, _ptr(q, torch.float64, "q"), _ptr(dqdt, torch.float64, "dqdt"),
                           None, 0, _stream(stream)))


def nn_train_step(model, x, y, lr=1e-3, loss=None, idx=None, stream=None):
    """One Adam step on rows idx of (x, y) (all rows when idx is None)."""
    batch = x.shape[0] if idx is None else idx.shape[0]
    if idx is not None and (idx.dtype != torch.int32 or not idx.is_cuda):
        raise ValueError("idx must be a device int32 tensor")
    need = lib().nn_train_ws(model.handle, batch)
    if model.train_ws is None or model.train_ws.numel() < need:
        model.train_ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    check(lib().nn_train_step(model.handle, _ptr(x, torch.float32, "x"), _ptr(y, torch.float32, "y"),
                              _ptr(idx, torch.int32, "idx"), batch, float(lr), _ptr(loss, torch.float32, "loss"),
                              _ptr(model.train_ws), model.train_ws.numel(), _stream(stream)))


def nn_data_stats(x, y, n_p, stream=None):
    """[mu_x(5), sigma_x(5), mu_y(5), sigma_y(5)] of a training set."""
    rows = x.shape[0]
    ws = torch.empty(lib().nn_stats_ws(rows), dtype=torch.uint8, device=x.device)
    out = (ctypes.c_double * 20)()
    check(lib().nn_data_stats(_ptr(x, torch.float32, "x"), _ptr(y, torch.float32, "y"), rows, n_p, out, _ptr(ws),
                              ws.numel(), _stream(stream)))
    return list(out)


def nn_column_stats(x, y, n_p, stream=None):
    """Device float64 tensor [4, 5 n_p]: per-column mu_x, sigma_x, mu_y, sigma_y."""
    rows = x.shape[0]
    ws = torch.empty(max(1, lib().nn_column_stats_ws(rows, n_p)), dtype=torch.uint8, device=x.device)
    out = torch.empty((4, 5 * n_p), dtype=torch.float64, device=x.device)
    check(lib().nn_column_stats(_ptr(x, torch.float32, "x"), _ptr(y, torch.float32, "y"), rows, n_p,
                                _ptr(out, torch.float64, "out"), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def solve_footprint(P, N, use_nn=False):
    return lib().solve_footprint(P, N, 1 if use_nn else 0)


class Server:
    """solve_server handle over a caller-owned device arena."""

    def __init__(self, arena_bytes, max_slots=64, device="cuda"):
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(lib().solve_server_create(_ptr(self.arena), arena_bytes, max_slots, ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, Re, P, N, t_end, use_nn=False, model=None, ke_every=1, ke_capacity=0, Cs=0.0, Mach=0.1,
               want_state=False, after_step=False):
        """after_step: with use_nn, Algorithm 1's correction after each step
        instead of the forcing at every stage."""
        import numpy as np
        r = solve_request()
        r.Re, r.t_end, r.Mach, r.Cs = Re, t_end, Mach, Cs
        r.P, r.N, r.use_nn, r.ke_every = P, N, 1 if use_nn else 0, ke_every
        r.model = model.handle if model is not None else None
        ke = np.zeros(2 * max(ke_capacity, 1))
        qout = np.zeros(5 * N ** 3 * (P + 1) ** 3) if want_state else None
        r.ke_host = ke.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if ke_capacity > 0 else None
        r.ke_capacity = ke_capacity
        r.nn_after_step = 1 if after_step else 0
        r.q_out_host = qout.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_state else None
        rid = ctypes.c_uint64()
        check(lib().solve_submit(self.handle, ctypes.byref(r), ctypes.byref(rid)))
        self._keep[rid.value] = (ke, qout, model)
        return rid.value

    def poll(self, rid):
        st = solve_status()
        rc = check(lib().solve_poll(self.handle, rid, ctypes.byref(st)), allow=(DG_EAGAIN,))
        return rc, st

    def results(self, rid):
        ke, qout, _ = self._keep[rid]
        return ke, qout

    def inject_nan(self, rid):
        check(lib().solve_inject_nan(self.handle, rid))

    def drain(self):
        check(lib().solve_server_drain(self.handle))

    def stats(self):
        busy, batches = ctypes.c_double(), ctypes.c_int64()
        check(lib().solve_server_stats(self.handle, ctypes.byref(busy), ctypes.byref(batches)))
        return busy.value, batches.value

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.solve_server_free(self.handle)
            self.handle = None

    def __del__(self):
        self.close()
