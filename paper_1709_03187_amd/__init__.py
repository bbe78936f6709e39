"""Python binding of libaco.so, the MI355X ACO hot-path library.

Argument marshalling only: every step runs in the library's HIP kernels.  The
functions keep the C entry points' names; arrays are torch tensors on the GPU
(their `data_ptr()` is passed through) and the stream defaults to torch's
current stream.  `Colony` is a convenience holder that allocates the device
buffers of one instance with torch and calls the entry points in order.

The library must have been built (`python -m paper_1709_03187_amd.build`);
importing a function that needs it raises if `libaco.so` is missing -- there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaco.so")
_lib = None

ACO_OK = 0
ACO_ERR_INVALID_ARG = -1
ACO_ERR_UNSUPPORTED = -2
ACO_ERR_DEGENERATE = -3
ACO_ERR_WORKSPACE = -4
ACO_ERR_HIP = -5
ACO_ERR_DEVICE = -6
ACO_COORD_LIMIT = 2**29 - 1
ACO_MAX_K = 64
NO_SLOT = 255

EXPORTS = (
    "aco_strerror", "aco_last_error", "aco_version", "aco_device_error", "aco_grid_bytes",
    "aco_build_candidates",
    "aco_init_pheromone", "aco_construct_workspace_bytes", "aco_construct_tours",
    "aco_update_workspace_bytes", "aco_update_pheromone", "aco_track_best",
    "aco_run_workspace_bytes", "aco_run", "aco_batch_workspace_bytes", "aco_batch_layout",
    "aco_batch_setup", "aco_batch_iterate", "aco_run_batched", "aco_features_workspace_bytes",
    "aco_edge_features", "aco_mlp_forward", "aco_mlp_backward_workspace_bytes",
    "aco_mlp_backward", "aco_mlp_adam", "aco_mlp_train", "aco_tour_edge_labels",
    "aco_construct_partial",
    "aco_update_local_best", "aco_pheromone_local_best", "aco_construct_ex",
    "aco_two_opt_workspace_bytes", "aco_two_opt", "aco_update_pheromone_static",
    "aco_workspace_bytes",
)
ACO_WS_GRID, ACO_WS_CONSTRUCT, ACO_WS_UPDATE, ACO_WS_RUN = 0, 1, 2, 3
ACO_WS_TWO_OPT, ACO_WS_FEATURES, ACO_WS_MLP_BACKWARD = 4, 5, 6
ACO_UPDATE_STATIC_BYTES = 32 << 20
ACO_TWO_OPT_MAX_WINDOW = 2048
ACO_SAMPLER_ROULETTE = 0
ACO_SAMPLER_INDEPENDENT = 1
ACO_MLP_PARAMS = 4801
ACO_MLP_OUT_LOGIT = 0
ACO_MLP_OUT_ETA_B = 1
ACO_ETA_DISTANCE = 0
ACO_ETA_LEARNED = 1
ACO_VIS_BITS = 1
ACO_VIS_BYTES = 2
ACO_VIS_BITS_X4 = 3


class AcoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class AcoParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("m", C.c_int32), ("k", C.c_int32),
                ("alpha", C.c_double), ("beta", C.c_double), ("rho", C.c_double),
                ("iterations", C.c_int32), ("deposit_shift", C.c_int32), ("seed", C.c_uint64),
                ("eta_mode", C.c_int32), ("mlp_w", C.c_void_p)]

    def __init__(self, *args, **kw):
        super().__init__(C.sizeof(AcoParams), *args, **kw)


class AcoConstructOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("sampler", C.c_int32), ("p_partial", C.c_double),
                ("max_modify", C.c_int32), ("lbest", C.c_void_p), ("lbest_len", C.c_void_p)]

    def __init__(self, *args, **kw):
        super().__init__(C.sizeof(AcoConstructOpts), *args, **kw)


class AcoTwoOptStats(C.Structure):
    _fields_ = [("selected", C.c_int32), ("converged", C.c_int32), ("rounds", C.c_int64),
                ("moves", C.c_int64), ("gain", C.c_int64)]


class AcoBatchLayout(C.Structure):
    _fields_ = [(f, C.c_size_t) for f in ("nn", "nnd", "rev", "eta_b", "tau", "tours", "slots",
                                          "lengths", "total")]


def lib():
    """Load libaco.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  -- loads the HIP runtime the library binds to
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1709_03187_amd.build")
        L = C.CDLL(LIB_PATH)
        p, i32, i64, u64, dbl, sz = (C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double,
                                     C.c_size_t)
        sig = {
            "aco_strerror": (C.c_char_p, [C.c_int]),
            "aco_last_error": (C.c_char_p, []),
            "aco_version": (C.c_char_p, []),
            "aco_device_error": (C.c_int, [p]),
            "aco_grid_bytes": (sz, [i32]),
            "aco_workspace_bytes": (sz, [i32, i32, i32, i32]),
            "aco_build_candidates": (C.c_int, [p, i32, i32, dbl, p, p, p, p, p, p, sz, p]),
            "aco_init_pheromone": (C.c_int, [p, i32, i32, p, p, p, p, p, p, p, p]),
            "aco_construct_workspace_bytes": (sz, [i32, i32]),
            "aco_construct_tours": (C.c_int, [p, i32, i32, p, p, p, p, p, i32, i32, dbl, u64,
                                              i64, p, p, p, p, p, sz, p]),
            "aco_update_workspace_bytes": (sz, [i32, i32, i32]),
            "aco_update_pheromone": (C.c_int, [i32, i32, p, p, i32, p, p, p, dbl, i32, p, p, sz,
                                               p]),
            "aco_update_pheromone_static": (C.c_int, [i32, i32, p, p, i32, p, p, p, dbl, i32,
                                                      p, p]),
            "aco_track_best": (C.c_int, [i32, i32, p, p, p, p, p, p]),
            "aco_run_workspace_bytes": (sz, [i32, C.POINTER(AcoParams)]),
            "aco_run": (C.c_int, [p, i32, C.POINTER(AcoParams), p, p, p, p, p, sz, p]),
            "aco_batch_workspace_bytes": (sz, [p, i32, C.POINTER(AcoParams)]),
            "aco_batch_layout": (C.c_int, [p, i32, C.POINTER(AcoParams),
                                           C.POINTER(AcoBatchLayout)]),
            "aco_batch_setup": (C.c_int, [p, p, i32, C.POINTER(AcoParams), p, p, p, sz, p]),
            "aco_batch_iterate": (C.c_int, [p, p, i32, C.POINTER(AcoParams), i32, i32, i32, i32,
                                            i32, p, p, p, p, p, sz, p]),
            "aco_run_batched": (C.c_int, [p, p, i32, C.POINTER(AcoParams), i32, p, p, p, p, sz,
                                          p, p]),
            "aco_features_workspace_bytes": (sz, []),
            "aco_edge_features": (C.c_int, [p, i32, i32, p, p, p, p, p, sz, p]),
            "aco_mlp_forward": (C.c_int, [p, i64, p, i32, dbl, p, p]),
            "aco_mlp_backward_workspace_bytes": (sz, [i64]),
            "aco_mlp_backward": (C.c_int, [p, p, i64, p, C.c_float, p, p, p, sz, p]),
            "aco_mlp_adam": (C.c_int, [p, p, p, p, i32, C.c_float, C.c_float, C.c_float,
                                       C.c_float, p]),
            "aco_mlp_train": (C.c_int, [p, p, C.c_int64, p, p, p, C.c_float, i32, i32,
                                        C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float,
                                        p, p, p, sz, p]),
            "aco_tour_edge_labels": (C.c_int, [i32, i32, p, p, p, p, p]),
            "aco_construct_partial": (C.c_int, [p, i32, i32, p, p, p, p, p, i32, i32, dbl, u64,
                                                i64, dbl, i32, p, p, p, p, p, p, sz, p]),
            "aco_update_local_best": (C.c_int, [i32, i32, p, p, p, p, p]),
            "aco_pheromone_local_best": (C.c_int, [i32, i32, p, p, i32, p, p, dbl, dbl, i32, p, p,
                                                   sz, p]),
            "aco_construct_ex": (C.c_int, [p, i32, i32, p, p, p, p, p, i32, i32, dbl, u64, i64,
                                           C.POINTER(AcoConstructOpts), p, p, p, p, p, sz, p]),
            "aco_two_opt_workspace_bytes": (sz, [i32, i32, i32]),
            "aco_two_opt": (C.c_int, [p, i32, i32, p, p, p, i32, dbl, u64, i64, i64, i32,
                                      C.POINTER(AcoTwoOptStats), p, sz, p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != ACO_OK:
        L = lib()
        raise AcoError(rc, f"{L.aco_strerror(rc).decode()}: {L.aco_last_error().decode()}")


def _ptr(t, dtype=None, name="array"):
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _t():
    import torch
    return torch


# ------------------------------------------------------------ entry points
def aco_version() -> str:
    return lib().aco_version().decode()


def aco_device_error(stream=None):
    """Synchronise and raise AcoError (ACO_ERR_DEVICE) if a kernel's device-side
    check failed since the last report."""
    _check(lib().aco_device_error(_stream(stream)))


def aco_workspace_bytes(which: int, n: int, k: int, m: int) -> int:
    return int(lib().aco_workspace_bytes(int(which), int(n), int(k), int(m)))


def aco_grid_bytes(n: int) -> int:
    return int(lib().aco_grid_bytes(n))


def aco_construct_workspace_bytes(n: int, k: int) -> int:
    return int(lib().aco_construct_workspace_bytes(n, k))


def aco_update_workspace_bytes(n: int, k: int, m: int) -> int:
    return int(lib().aco_update_workspace_bytes(n, k, m))


def aco_run_workspace_bytes(n: int, params: AcoParams) -> int:
    return int(lib().aco_run_workspace_bytes(n, C.byref(params)))


def aco_build_candidates(xy, n, k, beta, eta, nn, nnd, rev, eta_b, grid, stream=None):
    torch = _t()
    _check(lib().aco_build_candidates(
        _ptr(xy, torch.int32, "xy"), n, k, float(beta), _ptr(eta, torch.float32, "eta"),
        _ptr(nn, torch.int32, "nn"), _ptr(nnd, torch.int32, "nnd"), _ptr(rev, torch.int8, "rev"),
        _ptr(eta_b, torch.float32, "eta_b"), _ptr(grid, torch.uint8, "grid"), grid.numel(),
        _stream(stream)))


def aco_init_pheromone(xy, n, k, nn, nnd, grid, nn_tour, tau, stream=None):
    """Returns (tau0, L_nn)."""
    torch = _t()
    t0 = C.c_float(0)
    L = C.c_int64(0)
    _check(lib().aco_init_pheromone(
        _ptr(xy, torch.int32, "xy"), n, k, _ptr(nn, torch.int32, "nn"),
        _ptr(nnd, torch.int32, "nnd"), _ptr(grid, torch.uint8, "grid"),
        _ptr(nn_tour, torch.int32, "nn_tour"), _ptr(tau, torch.float32, "tau"), C.byref(t0),
        C.byref(L), _stream(stream)))
    return t0.value, L.value


def aco_construct_tours(xy, n, k, nn, nnd, eta_b, grid, tau, m, ant0, alpha, seed, iteration,
                        tours, lengths, slots, step_prob, ws, stream=None):
    torch = _t()
    _check(lib().aco_construct_tours(
        _ptr(xy, torch.int32, "xy"), n, k, _ptr(nn, torch.int32, "nn"),
        _ptr(nnd, torch.int32, "nnd"), _ptr(eta_b, torch.float32, "eta_b"),
        _ptr(grid, torch.uint8, "grid"), _ptr(tau, torch.float32, "tau"), m, ant0, float(alpha),
        int(seed), int(iteration), _ptr(tours, torch.int32, "tours"),
        _ptr(lengths, torch.int64, "lengths"), _ptr(slots, torch.uint8, "slots"),
        _ptr(step_prob, torch.float32, "step_prob"), _ptr(ws, torch.uint8, "ws"), ws.numel(),
        _stream(stream)))


def aco_update_pheromone(n, k, nn, rev, m, tours, slots, lengths, rho, deposit_shift, tau, ws,
                         stream=None):
    torch = _t()
    _check(lib().aco_update_pheromone(
        n, k, _ptr(nn, torch.int32, "nn"), _ptr(rev, torch.int8, "rev"), m,
        _ptr(tours, torch.int32, "tours"), _ptr(slots, torch.uint8, "slots"),
        _ptr(lengths, torch.int64, "lengths"), float(rho), int(deposit_shift),
        _ptr(tau, torch.float32, "tau"), _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream(stream)))


def aco_update_pheromone_static(n, k, nn, rev, m, tours, slots, lengths, rho, deposit_shift, tau,
                                stream=None):
    """aco_update_pheromone on the library's own per-device scratch (no workspace)."""
    torch = _t()
    _check(lib().aco_update_pheromone_static(
        n, k, _ptr(nn, torch.int32, "nn"), _ptr(rev, torch.int8, "rev"), m,
        _ptr(tours, torch.int32, "tours"), _ptr(slots, torch.uint8, "slots"),
        _ptr(lengths, torch.int64, "lengths"), float(rho), int(deposit_shift),
        _ptr(tau, torch.float32, "tau"), _stream(stream)))


def aco_track_best(n, m, tours, lengths, best_len, best_tour, iter_best=None, stream=None):
    torch = _t()
    _check(lib().aco_track_best(
        n, m, _ptr(tours, torch.int32, "tours"), _ptr(lengths, torch.int64, "lengths"),
        _ptr(best_len, torch.int64, "best_len"), _ptr(best_tour, torch.int32, "best_tour"),
        _ptr(iter_best, torch.int64, "iter_best"), _stream(stream)))


def aco_run(xy, n, params: AcoParams, best_tour, best_len, iter_best, tau_out, ws, stream=None):
    torch = _t()
    _check(lib().aco_run(
        _ptr(xy, torch.int32, "xy"), n, C.byref(params), _ptr(best_tour, torch.int32, "best_tour"),
        _ptr(best_len, torch.int64, "best_len"), _ptr(iter_best, torch.int64, "iter_best"),
        _ptr(tau_out, torch.float32, "tau_out"), _ptr(ws, torch.uint8, "ws"), ws.numel(),
        _stream(stream)))


def aco_construct_partial(xy, n, k, nn, nnd, eta_b, grid, tau, m, ant0, alpha, seed, iteration,
                          p_partial, max_modify, lbest, tours, lengths, slots, step_prob, ws,
                          stream=None):
    torch = _t()
    _check(lib().aco_construct_partial(
        _ptr(xy, torch.int32, "xy"), n, k, _ptr(nn, torch.int32, "nn"),
        _ptr(nnd, torch.int32, "nnd"), _ptr(eta_b, torch.float32, "eta_b"),
        _ptr(grid, torch.uint8, "grid"), _ptr(tau, torch.float32, "tau"), m, ant0, float(alpha),
        int(seed), int(iteration), float(p_partial), int(max_modify),
        _ptr(lbest, torch.int32, "lbest"), _ptr(tours, torch.int32, "tours"),
        _ptr(lengths, torch.int64, "lengths"), _ptr(slots, torch.uint8, "slots"),
        _ptr(step_prob, torch.float32, "step_prob"), _ptr(ws, torch.uint8, "ws"), ws.numel(),
        _stream(stream)))


def aco_construct_ex(xy, n, k, nn, nnd, eta_b, grid, tau, m, ant0, alpha, seed, iteration, sampler,
                     p_partial, max_modify, lbest, tours, lengths, slots, step_prob, ws,
                     stream=None, lbest_len=None):
    torch = _t()
    opts = AcoConstructOpts(int(sampler), float(p_partial), int(max_modify),
                            None if lbest is None else _ptr(lbest, torch.int32, "lbest").value,
                            None if lbest_len is None
                            else _ptr(lbest_len, torch.int64, "lbest_len").value)
    _check(lib().aco_construct_ex(
        _ptr(xy, torch.int32, "xy"), n, k, _ptr(nn, torch.int32, "nn"),
        _ptr(nnd, torch.int32, "nnd"), _ptr(eta_b, torch.float32, "eta_b"),
        _ptr(grid, torch.uint8, "grid"), _ptr(tau, torch.float32, "tau"), m, ant0, float(alpha),
        int(seed), int(iteration), C.byref(opts), _ptr(tours, torch.int32, "tours"),
        _ptr(lengths, torch.int64, "lengths"), _ptr(slots, torch.uint8, "slots"),
        _ptr(step_prob, torch.float32, "step_prob"), _ptr(ws, torch.uint8, "ws"), ws.numel(),
        _stream(stream)))


def aco_update_local_best(n, m, tours, lengths, lbest, lbest_len, stream=None):
    torch = _t()
    _check(lib().aco_update_local_best(
        n, m, _ptr(tours, torch.int32, "tours"), _ptr(lengths, torch.int64, "lengths"),
        _ptr(lbest, torch.int32, "lbest"), _ptr(lbest_len, torch.int64, "lbest_len"),
        _stream(stream)))


def aco_pheromone_local_best(n, k, nn, rev, m, lbest, lbest_len, tau_base, delta, deposit_shift,
                             tau, ws, stream=None):
    torch = _t()
    _check(lib().aco_pheromone_local_best(
        n, k, _ptr(nn, torch.int32, "nn"), _ptr(rev, torch.int8, "rev"), m,
        _ptr(lbest, torch.int32, "lbest"), _ptr(lbest_len, torch.int64, "lbest_len"),
        float(tau_base), float(delta), int(deposit_shift), _ptr(tau, torch.float32, "tau"),
        _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream(stream)))


def aco_two_opt_workspace_bytes(n, m, batch) -> int:
    return int(lib().aco_two_opt_workspace_bytes(int(n), int(m), int(batch)))


def aco_two_opt(xy, n, m, tours, lengths, slots, window, p, seed, iteration, max_rounds, batch, ws,
                stream=None) -> dict:
    """Windowed 2-opt of the participating tours (in place); returns the call's statistics."""
    torch = _t()
    st = AcoTwoOptStats()
    _check(lib().aco_two_opt(
        _ptr(xy, torch.int32, "xy"), n, m, _ptr(tours, torch.int32, "tours"),
        _ptr(lengths, torch.int64, "lengths"), _ptr(slots, torch.uint8, "slots"), int(window),
        float(p), int(seed), int(iteration), int(max_rounds), int(batch), C.byref(st),
        _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream(stream)))
    return dict(selected=st.selected, converged=bool(st.converged), rounds=st.rounds,
                moves=st.moves, gain=st.gain)


# ------------------------------------------------------------ learned heuristic
def aco_features_workspace_bytes() -> int:
    return int(lib().aco_features_workspace_bytes())


def aco_edge_features(xy, n, k, nn, nnd, rev, feat, ws, stream=None):
    torch = _t()
    _check(lib().aco_edge_features(
        _ptr(xy, torch.int32, "xy"), n, k, _ptr(nn, torch.int32, "nn"),
        _ptr(nnd, torch.int32, "nnd"), _ptr(rev, torch.int8, "rev"),
        _ptr(feat, torch.float32, "feat"), _ptr(ws, torch.uint8, "ws"), ws.numel(),
        _stream(stream)))


def aco_mlp_forward(feat, E, theta, mode, beta, out, stream=None):
    torch = _t()
    _check(lib().aco_mlp_forward(
        _ptr(feat, torch.float32, "feat"), int(E), _ptr(theta, torch.float32, "theta"), int(mode),
        float(beta), _ptr(out, torch.float32, "out"), _stream(stream)))


def aco_mlp_backward_workspace_bytes(E: int) -> int:
    return int(lib().aco_mlp_backward_workspace_bytes(int(E)))


def aco_mlp_backward(feat, labels, E, theta, pos_weight, grad, loss, ws, stream=None):
    torch = _t()
    _check(lib().aco_mlp_backward(
        _ptr(feat, torch.float32, "feat"), _ptr(labels, torch.uint8, "labels"), int(E),
        _ptr(theta, torch.float32, "theta"), float(pos_weight), _ptr(grad, torch.float32, "grad"),
        _ptr(loss, torch.float64, "loss"), _ptr(ws, torch.uint8, "ws"), ws.numel(),
        _stream(stream)))


def aco_mlp_adam(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    torch = _t()
    f32 = torch.float32
    _check(lib().aco_mlp_adam(
        _ptr(theta, f32, "theta"), _ptr(m, f32, "m"), _ptr(v, f32, "v"), _ptr(grad, f32, "grad"),
        int(step), float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))


def aco_mlp_train(feat, labels, E, theta, m, v, pos_weight, first_step, steps, batch, lr, grad,
                  loss, ws, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    torch = _t()
    f32 = torch.float32
    _check(lib().aco_mlp_train(
        _ptr(feat, f32, "feat"), _ptr(labels, torch.uint8, "labels"), int(E),
        _ptr(theta, f32, "theta"), _ptr(m, f32, "m"), _ptr(v, f32, "v"), float(pos_weight),
        int(first_step), int(steps), int(batch), float(lr), float(beta1), float(beta2),
        float(eps), _ptr(grad, f32, "grad"), _ptr(loss, torch.float64, "loss"),
        _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream(stream)))


def aco_tour_edge_labels(n, k, nn, tour, labels, pos_ws, stream=None):
    torch = _t()
    _check(lib().aco_tour_edge_labels(
        n, k, _ptr(nn, torch.int32, "nn"), _ptr(tour, torch.int32, "tour"),
        _ptr(labels, torch.uint8, "labels"), _ptr(pos_ws, torch.int32, "pos_ws"),
        _stream(stream)))


# ------------------------------------------------------------ convenience holder
@dataclass
class Colony:
    """Device buffers of one instance plus the calls of one ACO run.

    xy: int32 [n, 2] coordinates (host numpy or GPU tensor)."""
    xy: object
    k: int
    m: int
    alpha: float = 1.0
    beta: float = 2.0
    rho: float = 0.1
    seed: int = 1
    deposit_shift: int = 32
    eta: object = None          # optional learned heuristic score, float32 [n, k] on GPU
    theta: object = None        # optional MLP parameters (float32 [ACO_MLP_PARAMS] on GPU)
    want_prob: bool = False
    device: str = "cuda"

    def __post_init__(self):
        torch = _t()
        xy = torch.as_tensor(self.xy, dtype=torch.int32)
        self.xy = xy.to(self.device).contiguous()
        n, k, m, dev = self.xy.shape[0], self.k, self.m, self.device
        self.n = n
        self.nn = torch.empty((n, k), dtype=torch.int32, device=dev)
        self.nnd = torch.empty((n, k), dtype=torch.int32, device=dev)
        self.rev = torch.empty((n, k), dtype=torch.int8, device=dev)
        self.eta_b = torch.empty((n, k), dtype=torch.float32, device=dev)
        self.grid = torch.empty(aco_grid_bytes(n), dtype=torch.uint8, device=dev)
        self.tau = torch.empty((n, k), dtype=torch.float32, device=dev)
        self.nn_tour = torch.empty(n, dtype=torch.int32, device=dev)
        self.cws = torch.empty(aco_construct_workspace_bytes(n, k), dtype=torch.uint8, device=dev)
        self.uws = torch.empty(aco_update_workspace_bytes(n, k, m), dtype=torch.uint8, device=dev)
        self.tours = torch.empty((m, n), dtype=torch.int32, device=dev)
        self.lengths = torch.empty(m, dtype=torch.int64, device=dev)
        self.slots = torch.empty((m, n), dtype=torch.uint8, device=dev)
        self.step_prob = (torch.empty((m, n), dtype=torch.float32, device=dev)
                          if self.want_prob else None)
        self.best_tour = torch.empty(n, dtype=torch.int32, device=dev)
        self.best_len = torch.empty(1, dtype=torch.int64, device=dev)
        self.tau0 = None
        self.L_nn = None

    def build_candidates(self, stream=None):
        aco_build_candidates(self.xy, self.n, self.k, self.beta, self.eta, self.nn, self.nnd,
                             self.rev, self.eta_b, self.grid, stream)
        if self.theta is not None:
            self.apply_learned_heuristic(self.theta, stream)

    def features(self, stream=None):
        """The 8 edge features [n, k, 8] (float32, GPU)."""
        torch = _t()
        feat = torch.empty((self.n, self.k, 8), dtype=torch.float32, device=self.device)
        ws = torch.empty(aco_features_workspace_bytes(), dtype=torch.uint8, device=self.device)
        aco_edge_features(self.xy, self.n, self.k, self.nn, self.nnd, self.rev, feat, ws, stream)
        return feat

    def apply_learned_heuristic(self, theta, stream=None):
        """Replace eta_b by sigmoid(MLP score)^beta (candidates must be built)."""
        feat = self.features(stream)
        aco_mlp_forward(feat, self.n * self.k, theta, ACO_MLP_OUT_ETA_B, self.beta, self.eta_b,
                        stream)

    def init_pheromone(self, stream=None):
        self.tau0, self.L_nn = aco_init_pheromone(self.xy, self.n, self.k, self.nn, self.nnd,
                                                  self.grid, self.nn_tour, self.tau, stream)
        self.best_tour.copy_(self.nn_tour)
        self.best_len.fill_(self.L_nn)

    def setup(self, stream=None):
        self.build_candidates(stream)
        self.init_pheromone(stream)

    def construct(self, iteration, stream=None, m=None, ant0=0):
        m = self.m if m is None else m
        aco_construct_tours(self.xy, self.n, self.k, self.nn, self.nnd, self.eta_b, self.grid,
                            self.tau, m, ant0, self.alpha, self.seed, iteration, self.tours,
                            self.lengths, self.slots, self.step_prob, self.cws, stream)

    def construct_partial(self, iteration, p_partial, max_modify, stream=None):
        """PartialACO construction from the ants' local bests (`self.lbest`)."""
        aco_construct_partial(self.xy, self.n, self.k, self.nn, self.nnd, self.eta_b, self.grid,
                              self.tau, self.m, 0, self.alpha, self.seed, iteration, p_partial,
                              max_modify, self.lbest, self.tours, self.lengths, self.slots,
                              self.step_prob, self.cws, stream)

    def construct_ex(self, iteration, sampler=ACO_SAMPLER_ROULETTE, p_partial=0.0, max_modify=1,
                     partial=False, stream=None, use_lbest_len=True):
        """Construction with a chosen sampler; partial=True rebuilds from the local bests
        (whose kept part's length then comes from their lengths, unless
        use_lbest_len is False)."""
        aco_construct_ex(self.xy, self.n, self.k, self.nn, self.nnd, self.eta_b, self.grid,
                         self.tau, self.m, 0, self.alpha, self.seed, iteration, sampler,
                         p_partial, max_modify, self.lbest if partial else None, self.tours,
                         self.lengths, self.slots,
                         self.step_prob if sampler == ACO_SAMPLER_ROULETTE else None, self.cws,
                         stream, lbest_len=self.lbest_len if partial and use_lbest_len else None)

    def update_local_best(self, stream=None):
        """Take this iteration's tours into the local bests where strictly shorter
        (allocates the local bests on first use)."""
        torch = _t()
        if getattr(self, "lbest", None) is None:
            self.lbest = torch.empty((self.m, self.n), dtype=torch.int32, device=self.device)
            self.lbest_len = torch.full((self.m,), 2**63 - 1, dtype=torch.int64,
                                        device=self.device)
        aco_update_local_best(self.n, self.m, self.tours, self.lengths, self.lbest,
                              self.lbest_len, stream)

    def pheromone_from_local_best(self, tau_base, delta, stream=None):
        """tau from the local best tours (no evaporation), replacing the table."""
        aco_pheromone_local_best(self.n, self.k, self.nn, self.rev, self.m, self.lbest,
                                 self.lbest_len, tau_base, delta, self.deposit_shift, self.tau,
                                 self.uws, stream)

    def two_opt(self, iteration, p=0.001, window=500, max_rounds=0, batch=8, stream=None):
        """Windowed 2-opt of the tours that take part this iteration (in place; lengths and
        construction records follow).  Returns the call's statistics."""
        torch = _t()
        need = aco_two_opt_workspace_bytes(self.n, self.m, batch)
        if getattr(self, "tws", None) is None or self.tws.numel() < need:
            self.tws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return aco_two_opt(self.xy, self.n, self.m, self.tours, self.lengths, self.slots, window,
                           p, self.seed, iteration, max_rounds, batch, self.tws, stream)

    def track_best(self, iter_best=None, stream=None):
        aco_track_best(self.n, self.m, self.tours, self.lengths, self.best_len, self.best_tour,
                       iter_best, stream)

    def update(self, stream=None, use_slots=True):
        aco_update_pheromone(self.n, self.k, self.nn, self.rev, self.m, self.tours,
                             self.slots if use_slots else None, self.lengths, self.rho,
                             self.deposit_shift, self.tau, self.uws, stream)

    def iterate(self, iteration, iter_best=None, stream=None):
        """One pass of the hot path: construction, best tracking, update."""
        self.construct(iteration, stream)
        self.track_best(iter_best, stream)
        self.update(stream)


# ------------------------------------------------------------ batched colonies
def _host_i64(a):
    import numpy as np
    arr = np.ascontiguousarray(a, dtype=np.int64)
    return arr, arr.ctypes.data_as(C.c_void_p)


def aco_batch_workspace_bytes(offsets, B, params: AcoParams) -> int:
    arr, ptr = _host_i64(offsets)
    return int(lib().aco_batch_workspace_bytes(ptr, B, C.byref(params)))


def aco_batch_layout(offsets, B, params: AcoParams) -> AcoBatchLayout:
    arr, ptr = _host_i64(offsets)
    out = AcoBatchLayout()
    _check(lib().aco_batch_layout(ptr, B, C.byref(params), C.byref(out)))
    return out


def aco_batch_setup(xy, offsets, B, params, best_tours, best_lens, ws, stream=None):
    torch = _t()
    arr, ptr = _host_i64(offsets)
    _check(lib().aco_batch_setup(
        _ptr(xy, torch.int32, "xy"), ptr, B, C.byref(params),
        _ptr(best_tours, torch.int32, "best_tours"), _ptr(best_lens, torch.int64, "best_lens"),
        _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream(stream)))


def aco_batch_iterate(xy, offsets, B, params, first_iteration, count, waves, vis_layout,
                      occupancy, best_tours, best_lens, iter_best, ws, stream=None,
                      step_prob=None):
    torch = _t()
    arr, ptr = _host_i64(offsets)
    _check(lib().aco_batch_iterate(
        _ptr(xy, torch.int32, "xy"), ptr, B, C.byref(params), int(first_iteration), int(count),
        int(waves), int(vis_layout), int(occupancy),
        _ptr(best_tours, torch.int32, "best_tours"), _ptr(best_lens, torch.int64, "best_lens"),
        _ptr(iter_best, torch.int64, "iter_best"), _ptr(step_prob, torch.float32, "step_prob"),
        _ptr(ws, torch.uint8, "ws"), ws.numel(), _stream(stream)))


def aco_run_batched(xy, offsets, B, params, autotune, best_tours, best_lens, iter_best, ws,
                    stream=None):
    """Returns the launch shape and k used: (waves, layout, occupancy, k)."""
    torch = _t()
    arr, ptr = _host_i64(offsets)
    tuned = (C.c_int32 * 4)()
    _check(lib().aco_run_batched(
        _ptr(xy, torch.int32, "xy"), ptr, B, C.byref(params), int(autotune),
        _ptr(best_tours, torch.int32, "best_tours"), _ptr(best_lens, torch.int64, "best_lens"),
        _ptr(iter_best, torch.int64, "iter_best"), _ptr(ws, torch.uint8, "ws"), ws.numel(),
        _stream(stream), tuned))
    return int(tuned[0]), int(tuned[1]), int(tuned[2]), int(tuned[3])


class Batch:
    """Device buffers of a batch of instances (xy int32 [N, 2], offsets int64 [B+1])."""

    def __init__(self, xy, offsets, k, m, alpha=1.0, beta=2.0, rho=0.1, seed=4, iterations=30,
                 deposit_shift=32, device="cuda"):
        torch = _t()
        import numpy as np
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.B = len(self.offsets) - 1
        self.N = int(self.offsets[-1])
        self.params = AcoParams(m=m, k=k, alpha=alpha, beta=beta, rho=rho, iterations=iterations,
                                deposit_shift=deposit_shift, seed=seed)
        self.xy = torch.as_tensor(xy, dtype=torch.int32).to(device).contiguous()
        self.ws = torch.empty(aco_batch_workspace_bytes(self.offsets, self.B, self.params),
                              dtype=torch.uint8, device=device)
        self.best_tours = torch.empty(self.N, dtype=torch.int32, device=device)
        self.best_lens = torch.empty(self.B, dtype=torch.int64, device=device)
        # k = 0 (k-auto, run() only): the layout is known once run() has chosen k
        self.layout = aco_batch_layout(self.offsets, self.B, self.params) if k > 0 else None

    def setup(self, stream=None):
        aco_batch_setup(self.xy, self.offsets, self.B, self.params, self.best_tours,
                        self.best_lens, self.ws, stream)

    def iterate(self, first, count, waves=0, layout=0, iter_best=None, stream=None, occupancy=0,
                step_prob=None):
        aco_batch_iterate(self.xy, self.offsets, self.B, self.params, first, count, waves, layout,
                          occupancy, self.best_tours, self.best_lens, iter_best, self.ws, stream,
                          step_prob=step_prob)

    def run(self, autotune=1, iter_best=None, stream=None):
        """Set-up and all iterations; returns (waves, layout, occupancy, k).  With
        k = 0 the chosen k is kept in params and the state views follow it."""
        tuned = aco_run_batched(self.xy, self.offsets, self.B, self.params, autotune,
                                self.best_tours, self.best_lens, iter_best, self.ws, stream)
        if self.params.k == 0:
            self.params.k = tuned[3]
            self.layout = aco_batch_layout(self.offsets, self.B, self.params)
        return tuned

    def view(self, name, dtype, count):
        """A tensor view of one state array inside the workspace."""
        torch = _t()
        off = getattr(self.layout, name)
        size = torch.tensor([], dtype=dtype).element_size()
        return self.ws[off:off + count * size].view(dtype)
