"""Thin Python binding of libbfvec (ctypes).

Argument marshalling only: every step of the filter runs inside the native
library (include/bfvec.h).  torch supplies device memory and streams.  The
binding fails loudly when the library has not been built; there is no
fallback implementation.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfvec.so")

BF_OK, BF_EINVAL, BF_ENOTSPD, BF_ENOMEM, BF_EDEVICE, BF_EUNSUPPORTED, BF_EBUSY, \
    BF_ETIMEDOUT = range(8)
(BF_REQ_QUEUED, BF_REQ_PREPARING, BF_REQ_RUNNING, BF_REQ_DONE, BF_REQ_FAILED,
 BF_REQ_CANCELLED) = range(6)
REQ_STATES = {BF_REQ_QUEUED: "queued", BF_REQ_PREPARING: "preparing", BF_REQ_RUNNING: "running",
              BF_REQ_DONE: "done", BF_REQ_FAILED: "failed", BF_REQ_CANCELLED: "cancelled"}
BF_FP32, BF_FP16, BF_BF16, BF_FP32_SPLIT = 0, 1, 2, 5
PRECISIONS = {"fp32": BF_FP32, "fp16": BF_FP16, "bf16": BF_BF16, "fp32_split": BF_FP32_SPLIT}
BF_SPATIAL_GAUSS, BF_SPATIAL_BOX, BF_SPATIAL_HAT, BF_SPATIAL_BOX3 = 0, 1, 2, 3
BF_SPATIAL_RUNSUM = 16
BF_WHITEN_EIG, BF_WHITEN_CHOL, BF_WHITEN_SYM = 0, 1, 2
BF_POLICY_SHARE, BF_POLICY_SHORTEST_FIRST = 0, 1
POLICIES = {"share": BF_POLICY_SHARE, "shortest": BF_POLICY_SHORTEST_FIRST}
WHITEN = {"eig": BF_WHITEN_EIG, "chol": BF_WHITEN_CHOL, "sym": BF_WHITEN_SYM}


def _whiten_mode(v):
    return WHITEN[v] if isinstance(v, str) else int(v)
SPATIAL = {"gauss": BF_SPATIAL_GAUSS, "box": BF_SPATIAL_BOX, "hat": BF_SPATIAL_HAT,
           "box3": BF_SPATIAL_BOX3}


def _spatial(v):
    """"gauss", "box", "hat", "box3", optionally with "+runsum" (the
    running-sum vertical pass, FP32), or the integer value."""
    if isinstance(v, str):
        name, _, flag = v.partition("+")
        if flag not in ("", "runsum"):
            raise ValueError(f"unknown spatial flag {flag!r}")
        return SPATIAL[name] | (BF_SPATIAL_RUNSUM if flag else 0)
    return int(v)

# Every symbol declared in include/bfvec.h.
EXPORTS = [
    "bf_opts_init", "bf_vec", "bf_vec_ex", "bf_vec_terms", "bf_whiten", "bf_whiten_mode",
    "bf_sample_terms", "bf_choose_N", "bf_minmax", "bf_direct", "bf_autotune",
    "bf_last_error", "bf_version",
    "bf_server_config_init", "bf_request_init", "bf_server_create", "bf_server_submit",
    "bf_server_poll", "bf_server_wait", "bf_server_drain", "bf_server_forget",
    "bf_server_get_stats", "bf_server_clock", "bf_server_destroy",
    "bf_plan_create", "bf_plan_execute", "bf_plan_destroy", "bf_vec_static", "bf_ubench",
]
UBENCH = {"mfma_f32": 0, "mfma_f16": 1, "valu_f32": 2, "trans_f32": 3, "lds_read": 4,
          "hbm_copy": 5, "mfma_f32_solo": 6, "overlap_f32": 7, "overlap_f16": 8}
BF_STATIC_SCRATCH_BYTES = 64 << 20


class BfError(RuntimeError):
    """A libbfvec call returned a nonzero status."""

    def __init__(self, code, msg):
        super().__init__(f"libbfvec error {code}: {msg}")
        self.code = code


class bf_opts(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("center", ctypes.c_int),
        ("tile_h", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("num_out", ctypes.c_void_p),
        ("z_out", ctypes.c_void_p),
        ("N_used", ctypes.c_int),
        ("time_kernel", ctypes.c_int),
        ("kernel_ms", ctypes.c_float),
        ("dedup", ctypes.c_int),
        ("K_used", ctypes.c_int),
        ("tile_h_used", ctypes.c_int),
        ("spatial", ctypes.c_int),
        ("whiten", ctypes.c_int),
        ("tile_w", ctypes.c_int),
        ("tile_w_used", ctypes.c_int),
        ("valu_only", ctypes.c_int),
        ("mfma_used", ctypes.c_int),
    ]


class bf_server_config(ctypes.Structure):
    _fields_ = [
        ("arena_bytes", ctypes.c_uint64),
        ("max_active", ctypes.c_int),
        ("max_queued", ctypes.c_int),
        ("streams", ctypes.c_int),
        ("depth", ctypes.c_int),
        ("quantum_us", ctypes.c_double),
        ("policy", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("graph_rounds", ctypes.c_int),
        ("reserved", ctypes.c_int * 5),
    ]


class bf_request(ctypes.Structure):
    _fields_ = [
        ("f", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("H", ctypes.c_int),
        ("W", ctypes.c_int),
        ("d", ctypes.c_int),
        ("pitch", ctypes.c_int),
        ("sigma_s", ctypes.c_double),
        ("C", ctypes.c_void_p),
        ("K", ctypes.c_int),
        ("N", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("precision", ctypes.c_int),
        ("center", ctypes.c_int),
        ("arrival", ctypes.c_double),
        ("dedup", ctypes.c_int),
        ("spatial", ctypes.c_int),
        ("whiten", ctypes.c_int),
        ("reserved", ctypes.c_int * 1),
        ("f_host", ctypes.c_void_p),
        ("out_host", ctypes.c_void_p),
    ]


class bf_request_status(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int),
        ("error", ctypes.c_int),
        ("N_used", ctypes.c_int),
        ("chunks", ctypes.c_int),
        ("arrival", ctypes.c_double),
        ("admitted", ctypes.c_double),
        ("started", ctypes.c_double),
        ("done", ctypes.c_double),
        ("message", ctypes.c_char * 128),
    ]


class bf_server_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("failed", ctypes.c_uint64),
        ("rounds", ctypes.c_uint64),
        ("launches", ctypes.c_uint64),
        ("workgroups", ctypes.c_uint64),
        ("arena_bytes", ctypes.c_uint64),
        ("arena_peak", ctypes.c_uint64),
        ("admitted", ctypes.c_int),
        ("queued", ctypes.c_int),
        ("model_scale", ctypes.c_float),
        ("reserved", ctypes.c_int * 5),
    ]


_lib = None


def lib():
    """Load libbfvec.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} not found: build it first (python -m paper_1605_02164_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, U64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
    L.bf_opts_init.argtypes = [ctypes.POINTER(bf_opts)]
    L.bf_opts_init.restype = None
    L.bf_vec.argtypes = [P, I, I, I, D, P, I, U64, P]
    L.bf_vec_ex.argtypes = [P, I, I, I, D, P, I, U64, P, ctypes.POINTER(bf_opts)]
    L.bf_vec_terms.argtypes = [P, I, I, I, D, P, P, I, P, ctypes.POINTER(bf_opts)]
    L.bf_vec_static.argtypes = [P, I, I, I, D, P, I, U64, P, ctypes.POINTER(bf_opts)]
    L.bf_whiten.argtypes = [I, P, P]
    L.bf_whiten_mode.argtypes = [I, P, I, P]
    L.bf_sample_terms.argtypes = [I, P, I, I, U64, I, P, P]
    L.bf_choose_N.argtypes = [I, P, P, P, I, ctypes.POINTER(I)]
    L.bf_minmax.argtypes = [P, I, I, I, P, P, P]
    L.bf_direct.argtypes = [P, I, I, I, D, P, P]
    L.bf_autotune.argtypes = [P, I, I, I, D, I, P, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_float)]
    L.bf_last_error.argtypes = []
    L.bf_last_error.restype = ctypes.c_char_p
    L.bf_version.argtypes = []
    L.bf_server_config_init.argtypes = [ctypes.POINTER(bf_server_config)]
    L.bf_server_config_init.restype = None
    L.bf_request_init.argtypes = [ctypes.POINTER(bf_request)]
    L.bf_request_init.restype = None
    L.bf_server_create.argtypes = [ctypes.POINTER(bf_server_config), ctypes.POINTER(P)]
    L.bf_server_submit.argtypes = [P, ctypes.POINTER(bf_request), ctypes.POINTER(U64)]
    L.bf_server_poll.argtypes = [P, U64, ctypes.POINTER(bf_request_status)]
    L.bf_server_wait.argtypes = [P, U64, D, ctypes.POINTER(bf_request_status)]
    L.bf_server_drain.argtypes = [P, D]
    L.bf_server_forget.argtypes = [P, U64]
    L.bf_server_get_stats.argtypes = [P, ctypes.POINTER(bf_server_stats)]
    L.bf_server_clock.argtypes = [P]
    L.bf_server_clock.restype = D
    L.bf_server_destroy.argtypes = [P]
    L.bf_plan_create.argtypes = [I, I, I, D, P, I, U64, ctypes.POINTER(bf_opts), ctypes.POINTER(P)]
    L.bf_plan_execute.argtypes = [P, P, P, P]
    L.bf_plan_destroy.argtypes = [P]
    L.bf_ubench.argtypes = [I, I, ctypes.POINTER(D)]
    for name in ("bf_vec", "bf_vec_ex", "bf_vec_static", "bf_vec_terms", "bf_whiten",
                 "bf_whiten_mode",
                 "bf_sample_terms",
                 "bf_choose_N", "bf_minmax", "bf_direct", "bf_autotune", "bf_version",
                 "bf_server_create",
                 "bf_server_submit", "bf_server_poll", "bf_server_wait", "bf_server_drain",
                 "bf_server_forget", "bf_server_get_stats", "bf_server_destroy",
                 "bf_plan_create", "bf_plan_execute", "bf_plan_destroy", "bf_ubench"):
        getattr(L, name).restype = I
    _lib = L
    return L


def _check(rc):
    if rc != BF_OK:
        raise BfError(rc, lib().bf_last_error().decode())


def _host_f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check_image(f, out):
    import torch
    if not (f.is_cuda and f.dtype == torch.float32 and f.dim() == 3 and f.is_contiguous()):
        raise ValueError("f must be a contiguous (H, W, d) float32 CUDA tensor")
    if out is None:
        out = torch.empty_like(f)
    elif not (out.is_cuda and out.dtype == torch.float32 and out.shape == f.shape
              and out.is_contiguous()):
        raise ValueError("out must be a contiguous float32 CUDA tensor shaped like f")
    return out


def make_opts(N=0, precision="fp32", center=True, tile_h=0, stream=None,
              num_out=None, z_out=None, time_kernel=False, dedup=False, spatial="gauss",
              whiten="eig", tile_w=0, valu_only=False):
    o = bf_opts()
    lib().bf_opts_init(ctypes.byref(o))
    o.N = int(N)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.center = 1 if center else 0
    o.tile_h = int(tile_h)
    o.stream = stream
    o.num_out = None if num_out is None else num_out.data_ptr()
    o.z_out = None if z_out is None else z_out.data_ptr()
    o.time_kernel = 1 if time_kernel else 0
    o.dedup = 1 if dedup else 0
    o.spatial = _spatial(spatial)
    o.whiten = _whiten_mode(whiten)
    o.tile_w = int(tile_w)
    o.valu_only = 1 if valu_only else 0
    return o


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def bf_vec(f, sigma_s, C, K, seed, out=None):
    """The filter on a (H, W, d) float32 CUDA tensor; synchronous, default
    options (automatic order, FP32).  Returns out."""
    out = _check_image(f, out)
    H, W, d = f.shape
    Ch = _host_f64(C, (d, d))
    _check(lib().bf_vec(f.data_ptr(), H, W, d, float(sigma_s), _ptr(Ch), int(K),
                        int(seed) & 0xFFFFFFFFFFFFFFFF, out.data_ptr()))
    return out


def bf_vec_ex(f, sigma_s, C, K, seed, out=None, N=0, precision="fp32", center=True,
              tile_h=0, stream=None, num_out=None, z_out=None, time_kernel=False,
              return_opts=False, dedup=False, spatial="gauss", whiten="eig", tile_w=0,
              valu_only=False):
    """The filter with options, queued on ``stream`` (torch stream; default:
    current stream).  Returns (out, N_used), or (out, opts) with
    ``return_opts`` (opts.kernel_ms holds the fused-kernel time when
    ``time_kernel`` is set; opts.K_used the number of kernel terms, fewer than
    K with ``dedup``; opts.tile_h_used / tile_w_used the strip shape).
    ``spatial``: "gauss" (default), "box", "hat", "box3"; ``whiten``: "eig"
    (default), "chol", "sym"; ``tile_w``: strip width 0 (auto), 16 or 32;
    ``valu_only``: both passes on the vector ALUs (no matrix cores)."""
    out = _check_image(f, out)
    H, W, d = f.shape
    Ch = _host_f64(C, (d, d))
    o = make_opts(N, precision, center, tile_h, _stream_handle(stream), num_out, z_out,
                  time_kernel, dedup, spatial, whiten, tile_w, valu_only)
    _check(lib().bf_vec_ex(f.data_ptr(), H, W, d, float(sigma_s), _ptr(Ch), int(K),
                           int(seed) & 0xFFFFFFFFFFFFFFFF, out.data_ptr(), ctypes.byref(o)))
    return (out, o) if return_opts else (out, o.N_used)


def bf_vec_static(f, sigma_s, C, K, seed, out=None, N=0, precision="fp32", center=True,
                  tile_h=0, stream=None, num_out=None, z_out=None, return_opts=False,
                  dedup=False, spatial="gauss", whiten="eig", tile_w=0, valu_only=False):
    """bf_vec_ex through the allocation-free entry point (library-owned static
    device scratch of BF_STATIC_SCRATCH_BYTES per GPU; calls that overlap on
    the device race).  Returns (out, N_used), or (out, opts)."""
    out = _check_image(f, out)
    H, W, d = f.shape
    Ch = _host_f64(C, (d, d))
    o = make_opts(N, precision, center, tile_h, _stream_handle(stream), num_out, z_out,
                  False, dedup, spatial, whiten, tile_w, valu_only)
    _check(lib().bf_vec_static(f.data_ptr(), H, W, d, float(sigma_s), _ptr(Ch), int(K),
                               int(seed) & 0xFFFFFFFFFFFFFFFF, out.data_ptr(), ctypes.byref(o)))
    return (out, o) if return_opts else (out, o.N_used)


def bf_vec_terms(f, sigma_s, w, weights=None, out=None, precision="fp32", center=True,
                 tile_h=0, stream=None, num_out=None, z_out=None, spatial="gauss", tile_w=0,
                 valu_only=False):
    """The filter with an explicit (K, d) float64 term table and optional
    weights.  Returns out."""
    out = _check_image(f, out)
    H, W, d = f.shape
    wh = _host_f64(w)
    if wh.ndim != 2 or wh.shape[1] != d:
        raise ValueError("w must be (K, d)")
    K = wh.shape[0]
    wt = None if weights is None else _host_f64(weights, (K,))
    o = make_opts(0, precision, center, tile_h, _stream_handle(stream), num_out, z_out,
                  spatial=spatial, tile_w=tile_w, valu_only=valu_only)
    _check(lib().bf_vec_terms(f.data_ptr(), H, W, d, float(sigma_s), _ptr(wh),
                              None if wt is None else _ptr(wt), K, out.data_ptr(),
                              ctypes.byref(o)))
    return out


def bf_whiten(C, mode="eig"):
    """Host whitening: W with W^T W = C^{-1} ("eig" of eq. (COB), "chol",
    "sym")."""
    Ch = _host_f64(C)
    d = Ch.shape[0]
    W = np.empty((d, d))
    _check(lib().bf_whiten_mode(d, _ptr(Ch), _whiten_mode(mode), _ptr(W)))
    return W


def bf_sample_terms(C, N, K, seed, whiten="eig"):
    """Host draws with the given whitening: returns (Y int32 (K, d),
    w float64 (K, d))."""
    Ch = _host_f64(C)
    d = Ch.shape[0]
    Y = np.empty((K, d), dtype=np.int32)
    w = np.empty((K, d))
    _check(lib().bf_sample_terms(d, _ptr(Ch), int(N), int(K),
                                 int(seed) & 0xFFFFFFFFFFFFFFFF, _whiten_mode(whiten),
                                 _ptr(Y), _ptr(w)))
    return Y, w


def bf_choose_N(C, lo, hi, whiten="eig"):
    """Host order rule from the covariance, the whitening mode and the
    per-channel extrema."""
    Ch = _host_f64(C)
    d = Ch.shape[0]
    lo32 = np.ascontiguousarray(np.asarray(lo, dtype=np.float32).reshape(d))
    hi32 = np.ascontiguousarray(np.asarray(hi, dtype=np.float32).reshape(d))
    N = ctypes.c_int(0)
    _check(lib().bf_choose_N(d, _ptr(Ch), _ptr(lo32), _ptr(hi32), _whiten_mode(whiten),
                             ctypes.byref(N)))
    return N.value


def bf_minmax(f, stream=None):
    """Per-channel (lo, hi) of a CUDA image, as float32 numpy arrays."""
    _check_image(f, None)
    H, W, d = f.shape
    lo = np.empty(d, dtype=np.float32)
    hi = np.empty(d, dtype=np.float32)
    _check(lib().bf_minmax(f.data_ptr(), H, W, d, _ptr(lo), _ptr(hi),
                           _stream_handle(stream)))
    return lo, hi


def bf_autotune(f, sigma_s, precision="fp32", stream=None):
    """Measure and record the fused kernel's fastest strip height for this
    image shape; returns (tile_h, ms_per_term)."""
    _check_image(f, None)
    H, W, d = f.shape
    th = ctypes.c_int(0)
    ms = ctypes.c_float(0.0)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().bf_autotune(f.data_ptr(), H, W, d, float(sigma_s), prec, _stream_handle(stream),
                             ctypes.byref(th), ctypes.byref(ms)))
    return th.value, ms.value


def bf_direct(f, sigma_s, C, out=None):
    """Direct GPU evaluation of eqs. (BF)/(normal) (exact Gaussian range kernel)."""
    out = _check_image(f, out)
    H, W, d = f.shape
    Ch = _host_f64(C, (d, d))
    _check(lib().bf_direct(f.data_ptr(), H, W, d, float(sigma_s), _ptr(Ch), out.data_ptr()))
    return out


def bf_ubench(probe, param=0):
    """A device probe of include/bfvec.h (bf_ubench): probe one of UBENCH's
    names, param the chains per wave/lane (matrix and FMA probes) or the copy
    size in MiB.  Returns the rate (TFLOP/s, tera-operations/s or TB/s)."""
    r = ctypes.c_double(0.0)
    _check(lib().bf_ubench(UBENCH[probe] if isinstance(probe, str) else int(probe), int(param),
                           ctypes.byref(r)))
    return r.value


class Plan:
    """A fixed-shape plan (bf_plan_* of the C ABI): the host work of
    bf_vec_ex done once for (H, W, d, sigma_s, C, K, seed, options), then one
    HIP graph launch per image.  ``N`` must be explicit."""

    def __init__(self, H, W, d, sigma_s, C, K, seed, N, precision="fp32", center=True,
                 tile_h=0, dedup=False, spatial="gauss", whiten="eig", tile_w=0,
                 valu_only=False):
        Ch = _host_f64(C, (d, d))
        o = make_opts(N, precision, center, tile_h, None, None, None, False, dedup, spatial,
                      whiten, tile_w, valu_only)
        h = ctypes.c_void_p()
        _check(lib().bf_plan_create(int(H), int(W), int(d), float(sigma_s), _ptr(Ch), int(K),
                                    int(seed) & 0xFFFFFFFFFFFFFFFF, ctypes.byref(o),
                                    ctypes.byref(h)))
        self._h = h
        self.shape = (int(H), int(W), int(d))
        self.N_used, self.K_used, self.tile_h_used = o.N_used, o.K_used, o.tile_h_used
        self.tile_w_used = o.tile_w_used
        self.mfma_used = o.mfma_used

    def __call__(self, f, out=None, stream=None):
        """Queue the filter of f into out on ``stream`` (default: current
        stream); returns out without waiting."""
        if self._h is None:
            raise RuntimeError("plan is closed")
        out = _check_image(f, out)
        if tuple(f.shape) != self.shape:
            raise ValueError(f"plan is for shape {self.shape}, got {tuple(f.shape)}")
        _check(lib().bf_plan_execute(self._h, f.data_ptr(), out.data_ptr(),
                                     _stream_handle(stream)))
        return out

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            _check(lib().bf_plan_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version():
    return lib().bf_version()


def _status_dict(st):
    return {"state": REQ_STATES.get(st.state, st.state), "error": st.error, "N_used": st.N_used,
            "chunks": st.chunks, "arrival": st.arrival, "admitted": st.admitted,
            "started": st.started, "done": st.done, "message": st.message.decode()}


def _image_view(f):
    """(pointer, H, W, d, pitch) of an (H, W, d) float32 tensor (CUDA or
    host) whose rows may be strided (e.g. a crop of a larger image)."""
    import torch
    if not (f.dtype == torch.float32 and f.dim() == 3):
        raise ValueError("f must be an (H, W, d) float32 tensor")
    H, W, d = f.shape
    s0, s1, s2 = f.stride()
    if not ((s2 == 1 or d == 1) and (s1 == d or W == 1) and s0 % d == 0 and s0 // d >= W):
        raise ValueError("f must have contiguous pixels and a row pitch that is a multiple of d")
    return f.data_ptr(), H, W, d, s0 // d


class Server:
    """Continuous-batching server on the current device (bf_server_* of the
    C ABI).  ``submit`` queues one request and returns its ticket; the
    tensors it was given are kept alive here until the request is forgotten
    or the server closed."""

    def __init__(self, arena_bytes=0, max_active=0, max_queued=0, streams=0, depth=0,
                 quantum_us=0.0, policy="share", autotune=False, graph_rounds=False):
        cfg = bf_server_config()
        lib().bf_server_config_init(ctypes.byref(cfg))
        cfg.arena_bytes = int(arena_bytes)
        cfg.max_active = int(max_active)
        cfg.max_queued = int(max_queued)
        cfg.streams = int(streams)
        cfg.depth = int(depth)
        cfg.quantum_us = float(quantum_us)
        cfg.policy = POLICIES[policy] if isinstance(policy, str) else int(policy)
        cfg.autotune = 1 if autotune else 0
        cfg.graph_rounds = 1 if graph_rounds else 0
        h = ctypes.c_void_p()
        _check(lib().bf_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._refs = {}

    def submit(self, f, sigma_s, C, K, seed, out=None, N=0, precision="fp16", center=True,
               arrival=0.0, dedup=False, spatial="gauss", whiten="eig"):
        """Queue the filter of ``f`` (see bf_vec_ex for the arguments);
        ``arrival`` is the server-clock time the request arrives (0: now).
        ``f`` is a CUDA tensor, or a host (CPU, preferably pinned) tensor that
        the server uploads itself; ``out`` a CUDA tensor or a host tensor the
        server downloads into (default: like ``f``).  Returns (ticket, out)."""
        import torch
        ptr, H, W, d, pitch = _image_view(f)
        host_in = not f.is_cuda
        if out is None:
            out = torch.empty((H, W, d), dtype=torch.float32, device=f.device,
                              pin_memory=host_in)
        elif not (out.dtype == torch.float32 and tuple(out.shape) == (H, W, d)
                  and out.is_contiguous()):
            raise ValueError("out must be a contiguous (H, W, d) float32 tensor")
        Ch = _host_f64(C, (d, d))
        r = bf_request()
        lib().bf_request_init(ctypes.byref(r))
        r.f, r.f_host = (None, ptr) if host_in else (ptr, None)
        r.out, r.out_host = (out.data_ptr(), None) if out.is_cuda else (None, out.data_ptr())
        r.H, r.W, r.d, r.pitch = H, W, d, pitch
        r.sigma_s = float(sigma_s)
        r.C = Ch.ctypes.data
        r.K, r.N = int(K), int(N)
        r.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        r.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        r.center = 1 if center else 0
        r.arrival = float(arrival)
        r.dedup = 1 if dedup else 0
        r.spatial = _spatial(spatial)
        r.whiten = _whiten_mode(whiten)
        t = ctypes.c_uint64()
        _check(lib().bf_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._refs[t.value] = (f, out)
        return t.value, out

    def poll(self, ticket):
        st = bf_request_status()
        _check(lib().bf_server_poll(self._h, ticket, ctypes.byref(st)))
        return _status_dict(st)

    def wait(self, ticket, timeout=-1.0):
        """Block until the request ends; returns its status dict (raises
        BfError on timeout)."""
        st = bf_request_status()
        _check(lib().bf_server_wait(self._h, ticket, float(timeout), ctypes.byref(st)))
        return _status_dict(st)

    def drain(self, timeout=-1.0):
        _check(lib().bf_server_drain(self._h, float(timeout)))

    def forget(self, ticket):
        _check(lib().bf_server_forget(self._h, ticket))
        self._refs.pop(ticket, None)

    def stats(self):
        s = bf_server_stats()
        _check(lib().bf_server_get_stats(self._h, ctypes.byref(s)))
        return {n: getattr(s, n) for n, _ in bf_server_stats._fields_ if n != "reserved"}

    def clock(self):
        return lib().bf_server_clock(self._h)

    def close(self):
        if self._h:
            _check(lib().bf_server_destroy(self._h))
            self._h = None
            self._refs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
