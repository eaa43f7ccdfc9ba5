"""ctypes binding of libsambaten.so (the gfx950 HIP library).

The binding only marshals arguments: every step of the update runs in the
library's kernels.  Function names follow the C ABI in include/sambaten.h.
torch is used for device buffers and streams only.

Raises RuntimeError at import when the library has not been built; there is
no fallback path.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsambaten.so")

(SBT_OK, SBT_E_INVALID, SBT_E_SHAPE, SBT_E_NOMEM, SBT_E_DEVICE, SBT_E_NUMERIC, SBT_E_STATE,
 SBT_E_BUSY) = range(8)
SBT_DENSE, SBT_COO = 0, 1
SBT_FLAG_LAMBDA_AVG = 1
SBT_P_F64, SBT_P_F32, SBT_P_BF16 = 0, 1, 2
SBT_SCHED_BATCHED, SBT_SCHED_PLAIN = 0, 1
SBT_TUNE_OFF, SBT_TUNE_ON, SBT_TUNE_CACHED, SBT_TUNE_FIXED = 0, 1, 2, 3
SBT_TUNE_SHAPES = 3
(SBT_K_MTTKRP_C, SBT_K_MTTKRP_AB, SBT_K_GATHER, SBT_K_UPDATE, SBT_K_COO_MTTKRP,
 SBT_K_ROW_SOLVE) = range(6)
(SBT_REP_AP, SBT_REP_BP, SBT_REP_CP, SBT_REP_LAMP, SBT_REP_PI, SBT_REP_VALID, SBT_REP_AT,
 SBT_REP_BT, SBT_REP_CT, SBT_REP_RNEW, SBT_REP_CC) = range(11)


class sbt_config(ctypes.Structure):
    _fields_ = [
        ("rank", ctypes.c_int32),
        ("repetitions", ctypes.c_int32),
        ("als_iters", ctypes.c_int32),
        ("init_iters", ctypes.c_int32),
        ("sample_factor", ctypes.c_int32 * 3),
        ("format", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("tensor_id", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("k_capacity", ctypes.c_int64),
        ("max_batch", ctypes.c_int64),
        ("nnz_capacity", ctypes.c_int64),
        ("getrank_runs", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("getrank_threshold", ctypes.c_double),
        ("persist_summaries", ctypes.c_int32),
        ("summary_refresh", ctypes.c_int32),
    ]


class SbtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_pd = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes)
_SIGS = {
    "sbt_init_dense": (ctypes.c_int, [ctypes.POINTER(sbt_config), _vp, _i64, _i64, _i64, _vp, _vp,
                                      _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "sbt_init_coo": (ctypes.c_int, [ctypes.POINTER(sbt_config), _vp, _vp, _vp, _vp, _i64, _i64,
                                    _i64, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "sbt_destroy": (None, [_vp]),
    "sbt_update_batch_dense": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "sbt_update_batch_coo": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp]),
    "sbt_get_shape": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                     ctypes.POINTER(_i64), ctypes.POINTER(_i32)]),
    "sbt_get_factors": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "sbt_fit": (ctypes.c_int, [_vp, _pd, _vp]),
    "sbt_fms": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _pd, _vp]),
    "sbt_get_batch_counter": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint32)]),
    "sbt_memory_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "sbt_save": (ctypes.c_int, [_vp, ctypes.c_char_p, _vp]),
    "sbt_load": (ctypes.c_int, [ctypes.c_char_p, _vp, ctypes.POINTER(_vp)]),
    "sbt_last_sample": (ctypes.c_int, [_vp, _i32, _i32, _vp, ctypes.POINTER(_i64)]),
    "sbt_last_rep": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i64, ctypes.POINTER(_i64)]),
    "sbt_mttkrp_dense": (ctypes.c_int, [_i32, _i32, _vp, _i64, _i64, _i64, _i32, _vp, _vp, _vp,
                                        _i32, _vp, _vp]),
    "sbt_mttkrp_dense_noalloc": (ctypes.c_int, [_i32, _i32, _vp, _i64, _i64, _i64, _i32, _vp, _vp,
                                                _vp, _i32, _vp, _vp]),
    "sbt_mttkrp_coo": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _i64, _i32, _vp, _vp,
                                      _vp, _i32, _i32, _vp, _vp]),
    "sbt_profile_enable": (ctypes.c_int, [_vp, _i32]),
    "sbt_profile_read": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i64), _pd, _pd]),
    "sbt_server_create": (ctypes.c_int, [_i32, _i64, _i64, ctypes.POINTER(_vp)]),
    "sbt_server_submit_dense": (ctypes.c_int, [_vp, _vp, _vp, _i64,
                                               ctypes.POINTER(ctypes.c_uint64)]),
    "sbt_server_submit_coo": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _i64, _i64,
                                             ctypes.POINTER(ctypes.c_uint64)]),
    "sbt_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(_i32),
                                       ctypes.POINTER(ctypes.c_int), _pd, _pd, _pd]),
    "sbt_server_drain": (ctypes.c_int, [_vp]),
    "sbt_server_destroy": (None, [_vp]),
    "sbt_nd_init_dense": (ctypes.c_int, [ctypes.POINTER(sbt_config), _i32, _vp, _vp, _vp, _vp,
                                         _vp, _vp, ctypes.POINTER(_vp)]),
    "sbt_nd_init_coo": (ctypes.c_int, [ctypes.POINTER(sbt_config), _i32, _vp, _vp, _vp, _vp,
                                       _i64, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "sbt_nd_update_batch_coo": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _vp]),
    "sbt_nd_get_shape": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), _vp, ctypes.POINTER(_i32)]),
    "sbt_nd_get_factor": (ctypes.c_int, [_vp, _i32, _vp, _vp]),
    "sbt_nd_get_lambda": (ctypes.c_int, [_vp, _vp, _vp]),
    "sbt_nd_last_rep": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _i64, ctypes.POINTER(_i64)]),
    "sbt_autotune_set": (ctypes.c_int, [_i32, _i32]),
    "sbt_autotune_clear": (ctypes.c_int, []),
    "sbt_autotune_count": (ctypes.c_int, [ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "sbt_autotune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "sbt_autotune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "sbt_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "sbt_last_error": (ctypes.c_char_p, [_vp]),
}

_lib = None


def load():
    """Load libsambaten.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1709_00668_amd.build`")
    # torch ships its own HIP runtime; loaded first, it is the one the
    # library's libamdhip64 dependency resolves to, so device pointers and
    # streams from torch are valid in the library's calls.  Loading the
    # library first would bind it to the system runtime and leave torch and
    # the library on two runtimes in one process.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return sorted(_SIGS)


def _check(status, handle=None, what="", global_msg=False):
    if status != SBT_OK:
        lib = load()
        msg = lib.sbt_status_str(status).decode()
        if handle or global_msg:
            detail = lib.sbt_last_error(handle if handle else None).decode()
            if detail:
                msg = f"{msg}: {detail}"
        raise SbtError(status, f"{what}: {msg}" if what else msg)


def _ptr(a):
    """Device or host address of a torch tensor / numpy array / int / None."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def make_config(rank, repetitions, als_iters, sample_factor, seed, *, init_iters=100,
                fmt=SBT_DENSE, precision=SBT_P_F32, schedule=SBT_SCHED_BATCHED, tensor_id=0,
                k_capacity, max_batch, nnz_capacity=0, getrank_runs=0,
                getrank_threshold=90.0, persist_summaries=False, summary_refresh=0, flags=0):
    c = sbt_config()
    c.rank, c.repetitions, c.als_iters, c.init_iters = rank, repetitions, als_iters, init_iters
    s = (sample_factor,) * 3 if np.isscalar(sample_factor) else tuple(sample_factor)
    for m in range(3):
        c.sample_factor[m] = int(s[m])
    c.format, c.precision, c.schedule = fmt, precision, schedule
    c.seed, c.tensor_id, c.flags = seed, tensor_id, flags
    c.k_capacity, c.max_batch, c.nnz_capacity = k_capacity, max_batch, nnz_capacity
    c.getrank_runs, c.reserved, c.getrank_threshold = getrank_runs, 0, getrank_threshold
    c.persist_summaries, c.summary_refresh = int(bool(persist_summaries)), summary_refresh
    return c


def coo_to_device(idx, vals):
    """(nnz, 3) integer coordinates and values -> ((i, j, k) int32, v float32) on device."""
    import torch
    idx = np.asarray(idx)
    cols = tuple(torch.from_numpy(np.ascontiguousarray(idx[:, m], dtype=np.int32)).cuda()
                 for m in range(3))
    v = torch.from_numpy(np.ascontiguousarray(vals, dtype=np.float32)).cuda()
    return cols, v


def dense_to_device(X, dtype):
    """(I, J, K) array -> device tensor whose memory is the column-major layout
    the library expects (torch shape (K, J, I), contiguous)."""
    import torch
    arr = np.ascontiguousarray(np.asarray(X, dtype=dtype).transpose(2, 1, 0))
    return torch.from_numpy(arr).cuda()


class Tensor:
    """Owning wrapper of an sbt_tensor handle."""

    def __init__(self, handle):
        self.h = handle

    # -- construction -------------------------------------------------------
    @classmethod
    def init_dense(cls, cfg, X0_dev, I, J, K0, factors=None, stream=None):
        lib = load()
        out = _vp()
        keep = []
        fa = [None] * 4
        if factors is not None:
            for q, f in enumerate(factors):
                a = np.ascontiguousarray(f, dtype=np.float64)
                keep.append(a)
                fa[q] = a.ctypes.data
        st = lib.sbt_init_dense(ctypes.byref(cfg), _ptr(X0_dev), I, J, K0, fa[0], fa[1], fa[2],
                                fa[3], _stream(stream), ctypes.byref(out))
        _check(st, None, "sbt_init_dense", global_msg=True)
        return cls(out.value)

    @classmethod
    def init_coo(cls, cfg, idx_dev, vals_dev, nnz, I, J, K0, factors=None, stream=None):
        """idx_dev: three int32 device arrays (i, j, k); vals_dev: float32.
        factors None: the initial decomposition is CP-ALS on the tensor."""
        lib = load()
        out = _vp()
        keep = [np.ascontiguousarray(f, dtype=np.float64) for f in (factors or ())]
        fa = [a.ctypes.data for a in keep] if keep else [None] * 4
        st = lib.sbt_init_coo(ctypes.byref(cfg), _ptr(idx_dev[0]), _ptr(idx_dev[1]),
                              _ptr(idx_dev[2]), _ptr(vals_dev), nnz, I, J, K0, fa[0], fa[1],
                              fa[2], fa[3], _stream(stream), ctypes.byref(out))
        _check(st, None, "sbt_init_coo", global_msg=True)
        return cls(out.value)

    @classmethod
    def load_file(cls, path, stream=None):
        """A tensor resumed from a checkpoint written by save()."""
        out = _vp()
        st = load().sbt_load(os.fsencode(path), _stream(stream), ctypes.byref(out))
        _check(st, None, "sbt_load", global_msg=True)
        return cls(out.value)

    def memory_bytes(self):
        """(resident, workspace) device bytes."""
        a, b = _i64(), _i64()
        _check(load().sbt_memory_bytes(self.h, ctypes.byref(a), ctypes.byref(b)), self.h,
               "sbt_memory_bytes")
        return a.value, b.value

    def save(self, path, stream=None):
        st = load().sbt_save(self.h, os.fsencode(path), _stream(stream))
        _check(st, self.h, "sbt_save")

    def close(self):
        if self.h:
            load().sbt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- update ---------------------------------------------------------------
    def update_batch_dense(self, Y_dev, K_new, stream=None):
        st = load().sbt_update_batch_dense(self.h, _ptr(Y_dev), K_new, _stream(stream))
        _check(st, self.h, "sbt_update_batch_dense")

    def update_batch_coo(self, idx_dev, vals_dev, nnz, K_new, stream=None):
        st = self.try_update_batch_coo(idx_dev, vals_dev, nnz, K_new, stream)
        _check(st, self.h, "sbt_update_batch_coo")

    def try_update_batch_coo(self, idx_dev, vals_dev, nnz, K_new, stream=None):
        return load().sbt_update_batch_coo(self.h, _ptr(idx_dev[0]), _ptr(idx_dev[1]),
                                           _ptr(idx_dev[2]), _ptr(vals_dev), nnz, K_new,
                                           _stream(stream))

    def try_update_batch_dense(self, Y_dev, K_new, stream=None):
        return load().sbt_update_batch_dense(self.h, _ptr(Y_dev), K_new, _stream(stream))

    # -- queries -------------------------------------------------------------
    def shape(self):
        I, J, K, R = _i64(), _i64(), _i64(), _i32()
        _check(load().sbt_get_shape(self.h, ctypes.byref(I), ctypes.byref(J), ctypes.byref(K),
                                    ctypes.byref(R)), self.h)
        return I.value, J.value, K.value, R.value

    def batch_counter(self):
        c = ctypes.c_uint32()
        _check(load().sbt_get_batch_counter(self.h, ctypes.byref(c)), self.h)
        return c.value

    def get_factors(self, stream=None):
        I, J, K, R = self.shape()
        A, B = np.empty((I, R)), np.empty((J, R))
        C, lam = np.empty((K, R)), np.empty(R)
        _check(load().sbt_get_factors(self.h, A.ctypes.data, B.ctypes.data, C.ctypes.data,
                                      lam.ctypes.data, _stream(stream)), self.h, "sbt_get_factors")
        return A, B, C, lam

    def fit(self, stream=None):
        f = ctypes.c_double()
        _check(load().sbt_fit(self.h, ctypes.byref(f), _stream(stream)), self.h, "sbt_fit")
        return f.value

    def fms(self, A, B, C, lam, stream=None):
        """Factor match score against a reference model (device tensors, or
        arrays copied to the device first), shapes as get_factors returns."""
        import torch
        I, J, K, R = self.shape()
        dev = []
        for M, shp in ((A, (I, R)), (B, (J, R)), (C, (K, R)), (lam, (R,))):
            t = M if isinstance(M, torch.Tensor) else torch.from_numpy(np.asarray(M))
            t = t.to(device="cuda", dtype=torch.float64).contiguous()
            if tuple(t.shape) != shp:
                raise ValueError(f"reference factor of shape {tuple(t.shape)}, expected {shp}")
            dev.append(t)
        f = ctypes.c_double()
        _check(load().sbt_fms(self.h, dev[0].data_ptr(), dev[1].data_ptr(), dev[2].data_ptr(),
                              dev[3].data_ptr(), ctypes.byref(f), _stream(stream)), self.h,
               "sbt_fms")
        return f.value

    def last_sample(self, rep, mode):
        I, J, K, R = self.shape()
        buf = np.empty(max(I, J, K) + 1, dtype=np.int32)
        n = _i64()
        _check(load().sbt_last_sample(self.h, rep, mode, buf.ctypes.data, ctypes.byref(n)),
               self.h, "sbt_last_sample")
        return buf[:n.value].copy()

    def profile_enable(self, on=True, every=1):
        """Kernel timing on/off; every=n times every n-th timed launch."""
        _check(load().sbt_profile_enable(self.h, int(every) if on else 0), self.h)

    def profile_read(self, kind):
        n, ms, b = _i64(), ctypes.c_double(), ctypes.c_double()
        _check(load().sbt_profile_read(self.h, kind, ctypes.byref(n), ctypes.byref(ms),
                                       ctypes.byref(b)), self.h)
        return n.value, ms.value, b.value

    def last_rep(self, rep, item, max_rows, ncols=None):
        """Debug copy of one repetition's item (rows x R, or rows x ncols for
        items with another width: 1 for SBT_REP_RNEW, getrank_runs for
        SBT_REP_CC)."""
        I, J, K, R = self.shape()
        nc = R if ncols is None else ncols
        cap = (max_rows + 1) * max(R, nc)
        buf = np.empty(cap)
        rows = _i64()
        _check(load().sbt_last_rep(self.h, rep, item, buf.ctypes.data, cap, ctypes.byref(rows)),
               self.h, "sbt_last_rep")
        return buf[:rows.value * nc].reshape(rows.value, nc).copy()


SBT_ND_REP_UP, SBT_ND_REP_UT, SBT_ND_REP_CT, SBT_ND_REP_LAMP, SBT_ND_REP_PI, SBT_ND_REP_VALID = \
    range(6)


def coo_nd_to_device(idx, vals):
    """(nnz, N) integer coordinates and values -> (N int32 coordinate arrays, float32
    values) on the device."""
    import torch
    idx = np.asarray(idx)
    cols = tuple(torch.from_numpy(np.ascontiguousarray(idx[:, m], dtype=np.int32)).cuda()
                 for m in range(idx.shape[1]))
    v = torch.from_numpy(np.ascontiguousarray(vals, dtype=np.float32)).cuda()
    return cols, v


def dense_nd_to_device(X, dtype):
    """Order-N array -> device tensor whose memory is the column-major layout
    the library expects (first index fastest)."""
    import torch
    X = np.asarray(X, dtype=dtype)
    arr = np.ascontiguousarray(X.transpose(tuple(range(X.ndim - 1, -1, -1))))
    return torch.from_numpy(arr).cuda()


class TensorN(Tensor):
    """An order-N tensor (sbt_nd_*); the last mode grows."""

    @classmethod
    def init_dense_nd(cls, cfg, X0_dev, dims, sample_factor, factors=None, lam=None,
                      stream=None):
        lib = load()
        N = len(dims)
        d = np.ascontiguousarray(dims, dtype=np.int64)
        s = (sample_factor,) * N if np.isscalar(sample_factor) else tuple(sample_factor)
        sf = np.ascontiguousarray(s, dtype=np.int32)
        keep = []
        fptr = None
        lptr = None
        if factors is not None:
            arrs = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
            keep.extend(arrs)
            fptr = (ctypes.c_void_p * N)(*[a.ctypes.data for a in arrs])
            la = np.ascontiguousarray(lam, dtype=np.float64)
            keep.append(la)
            lptr = la.ctypes.data
        out = _vp()
        st = lib.sbt_nd_init_dense(ctypes.byref(cfg), N, d.ctypes.data, sf.ctypes.data,
                                   _ptr(X0_dev), ctypes.cast(fptr, _vp) if fptr else None, lptr,
                                   _stream(stream), ctypes.byref(out))
        _check(st, None, "sbt_nd_init_dense", global_msg=True)
        return cls(out.value)

    @classmethod
    def init_coo_nd(cls, cfg, cols, v, dims, sample_factor, factors=None, lam=None,
                    stream=None):
        """cols: N device int32 coordinate arrays (the last inside 0..dims[-1]-1), v:
        device float32 values."""
        lib = load()
        N = len(dims)
        d = np.ascontiguousarray(dims, dtype=np.int64)
        s = (sample_factor,) * N if np.isscalar(sample_factor) else tuple(sample_factor)
        sf = np.ascontiguousarray(s, dtype=np.int32)
        nnz = int(v.numel())
        iptr = (ctypes.c_void_p * N)(*[_ptr(c) for c in cols])
        keep = []
        fptr = None
        lptr = None
        if factors is not None:
            arrs = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
            keep.extend(arrs)
            fptr = (ctypes.c_void_p * N)(*[a.ctypes.data for a in arrs])
            la = np.ascontiguousarray(lam, dtype=np.float64)
            keep.append(la)
            lptr = la.ctypes.data
        out = _vp()
        st = lib.sbt_nd_init_coo(ctypes.byref(cfg), N, d.ctypes.data, sf.ctypes.data,
                                 ctypes.cast(iptr, _vp), _ptr(v), nnz,
                                 ctypes.cast(fptr, _vp) if fptr else None, lptr,
                                 _stream(stream), ctypes.byref(out))
        _check(st, None, "sbt_nd_init_coo", global_msg=True)
        return cls(out.value)

    def update_batch_coo_nd(self, cols, v, K_new, stream=None):
        """cols: N device int32 coordinate arrays, the last batch-relative (0..K_new-1)."""
        iptr = (ctypes.c_void_p * len(cols))(*[_ptr(c) for c in cols])
        _check(load().sbt_nd_update_batch_coo(self.h, ctypes.cast(iptr, _vp), _ptr(v),
                                              int(v.numel()), int(K_new), _stream(stream)),
               self.h, "sbt_nd_update_batch_coo")

    def shape_nd(self):
        order, R = _i32(), _i32()
        dims = np.zeros(8, dtype=np.int64)
        _check(load().sbt_nd_get_shape(self.h, ctypes.byref(order), dims.ctypes.data,
                                       ctypes.byref(R)), self.h, "sbt_nd_get_shape")
        return [int(v) for v in dims[:order.value]], R.value

    def get_factors_nd(self, stream=None):
        dims, R = self.shape_nd()
        out = []
        for m, D in enumerate(dims):
            U = np.empty((D, R))
            _check(load().sbt_nd_get_factor(self.h, m, U.ctypes.data, _stream(stream)), self.h,
                   "sbt_nd_get_factor")
            out.append(U)
        lam = np.empty(R)
        _check(load().sbt_nd_get_lambda(self.h, lam.ctypes.data, _stream(stream)), self.h,
               "sbt_nd_get_lambda")
        return out, lam

    def last_sample(self, rep, mode):
        dims, R = self.shape_nd()
        buf = np.empty(max(dims) + 1, dtype=np.int32)
        n = _i64()
        _check(load().sbt_last_sample(self.h, rep, mode, buf.ctypes.data, ctypes.byref(n)),
               self.h, "sbt_last_sample")
        return buf[:n.value].copy()

    def last_rep_nd(self, rep, item, mode=0, max_rows=1 << 20):
        dims, R = self.shape_nd()
        cap = (max_rows + 1) * R
        buf = np.empty(cap)
        n = _i64()
        _check(load().sbt_nd_last_rep(self.h, rep, item, mode, buf.ctypes.data, cap,
                                      ctypes.byref(n)), self.h, "sbt_nd_last_rep")
        v = buf[:n.value].copy()
        return v if item in (SBT_ND_REP_LAMP, SBT_ND_REP_PI, SBT_ND_REP_VALID) else \
            v.reshape(-1, R)


def autotune_set(mode, shape=0):
    """Launch-shape tuner mode (process-wide): SBT_TUNE_OFF / ON / CACHED, or
    SBT_TUNE_FIXED with every tuned launch in `shape`."""
    _check(load().sbt_autotune_set(int(mode), int(shape)), None, "sbt_autotune_set")


def autotune_clear():
    _check(load().sbt_autotune_clear(), None, "sbt_autotune_clear")


def autotune_count():
    """(keys decided, keys with trials running)."""
    d, u = _i64(), _i64()
    _check(load().sbt_autotune_count(ctypes.byref(d), ctypes.byref(u)), None,
           "sbt_autotune_count")
    return d.value, u.value


def autotune_save(path):
    _check(load().sbt_autotune_save(os.fsencode(path)), None, "sbt_autotune_save")


def autotune_load(path):
    _check(load().sbt_autotune_load(os.fsencode(path)), None, "sbt_autotune_load")


def mttkrp_dense(precision, Z_dev, n1, n2, n3, R, U0_dev, U1_dev, U2_dev, mode, out_dev,
                 stream=None, schedule=SBT_SCHED_BATCHED):
    st = load().sbt_mttkrp_dense(precision, schedule, _ptr(Z_dev), n1, n2, n3, R, _ptr(U0_dev),
                                 _ptr(U1_dev), _ptr(U2_dev), mode, _ptr(out_dev), _stream(stream))
    _check(st, None, "sbt_mttkrp_dense")


def mttkrp_dense_noalloc(precision, Z_dev, n1, n2, n3, R, U0_dev, U1_dev, U2_dev, mode, out_dev,
                         stream=None, schedule=SBT_SCHED_BATCHED):
    """Enqueues only (no allocation, no synchronisation): the result is ready
    when `stream` reaches the launched kernels."""
    st = load().sbt_mttkrp_dense_noalloc(precision, schedule, _ptr(Z_dev), n1, n2, n3, R,
                                         _ptr(U0_dev), _ptr(U1_dev), _ptr(U2_dev), mode,
                                         _ptr(out_dev), _stream(stream))
    _check(st, None, "sbt_mttkrp_dense_noalloc")


def mttkrp_coo(idx_dev, vals_dev, nnz, n1, n2, n3, R, U0_dev, U1_dev, U2_dev, mode, out_dev,
               lanes=0, stream=None):
    """idx_dev: three int32 device arrays (a, b, c); vals_dev: float32."""
    st = load().sbt_mttkrp_coo(_ptr(idx_dev[0]), _ptr(idx_dev[1]), _ptr(idx_dev[2]),
                               _ptr(vals_dev), nnz, n1, n2, n3, R, _ptr(U0_dev), _ptr(U1_dev),
                               _ptr(U2_dev), mode, lanes, _ptr(out_dev), _stream(stream))
    _check(st, None, "sbt_mttkrp_coo")


class Server:
    """Serving loop over resident tensors (sbt_server_*)."""

    def __init__(self, slots, staging_bytes, hbm_budget_bytes=0):
        out = _vp()
        _check(load().sbt_server_create(slots, int(staging_bytes), int(hbm_budget_bytes),
                                        ctypes.byref(out)), None, "sbt_server_create")
        self.h = out.value

    def submit_dense(self, tensor, Y_dev, K_new):
        """Returns the ticket; raises on a request that can never be admitted."""
        tk = ctypes.c_uint64()
        st = load().sbt_server_submit_dense(self.h, tensor.h, _ptr(Y_dev), K_new,
                                            ctypes.byref(tk))
        _check(st, None, "sbt_server_submit_dense")
        return tk.value

    def try_submit_dense(self, tensor, Y_dev, K_new):
        tk = ctypes.c_uint64()
        st = load().sbt_server_submit_dense(self.h, tensor.h, _ptr(Y_dev), K_new,
                                            ctypes.byref(tk))
        return st, tk.value

    def submit_coo(self, tensor, idx_dev, vals_dev, nnz, K_new):
        """idx_dev: three int32 device arrays (i, j, k batch-relative); vals_dev: float32."""
        tk = ctypes.c_uint64()
        st = load().sbt_server_submit_coo(self.h, tensor.h, _ptr(idx_dev[0]), _ptr(idx_dev[1]),
                                          _ptr(idx_dev[2]), _ptr(vals_dev), nnz, K_new,
                                          ctypes.byref(tk))
        _check(st, None, "sbt_server_submit_coo")
        return tk.value

    def poll(self, ticket):
        """(state, result, t_submit, t_start, t_done)"""
        state, res = _i32(), ctypes.c_int()
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(load().sbt_server_poll(self.h, ticket, ctypes.byref(state), ctypes.byref(res),
                                      ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               None, "sbt_server_poll")
        return state.value, res.value, a.value, b.value, c.value

    def drain(self):
        _check(load().sbt_server_drain(self.h), None, "sbt_server_drain")

    def close(self):
        if self.h:
            load().sbt_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
