"""Build and load the C part of the oracle (test infrastructure only)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bmf_oracle.c")
_SO = os.path.join(_HERE, "liborc.so")

_lib = None


def build(force=True):
    """Compile bmf_oracle.c with gcc (plain -O2, IEEE FP64, OpenMP)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


_P = ctypes.POINTER
_d = ctypes.c_double
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_vp = ctypes.c_void_p


def lib():
    """Load liborc.so, building it first when it is missing or stale."""
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    L = ctypes.CDLL(_SO)
    L.orc_philox4x32_10.argtypes = [_vp, _vp, _vp]
    L.orc_philox4x32_10.restype = None
    L.orc_philox_batch.argtypes = [_i64, _vp, _u64, _vp]
    L.orc_philox_batch.restype = None
    L.orc_u23.argtypes = [_u32]
    L.orc_u23.restype = _d
    L.orc_normals.argtypes = [_u64, _u32, _u32, _u32, _i32, _vp]
    L.orc_normals.restype = None
    L.orc_gamma.argtypes = [_u64, _u32, _u32, _u32, _d]
    L.orc_gamma.restype = _d
    L.orc_cholesky.argtypes = [_i32, _vp, _vp]
    L.orc_cholesky.restype = ctypes.c_int
    L.orc_seq_mean.argtypes = [_i64, _vp]
    L.orc_seq_mean.restype = _d
    L.orc_init_side.argtypes = [_i64, _i32, _u64, _u32, _vp]
    L.orc_init_side.restype = None
    L.orc_update_side.argtypes = [_i64, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _d, _u64,
                                  _u32, _u32, _vp, _i32]
    L.orc_update_side.restype = _i64
    L.orc_cond_precision.argtypes = [_i64, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _d, _vp]
    L.orc_cond_precision.restype = None
    L.orc_sse.argtypes = [_i64, _i32, _vp, _vp, _vp, _vp, _vp]
    L.orc_sse.restype = _d
    L.orc_tau_draw.argtypes = [_d, _i64, _d, _d, _u64, _u32, _u32]
    L.orc_tau_draw.restype = _d
    L.orc_nw_draw.argtypes = [_i64, _i32, _vp, _vp, _d, _d, _vp, _u64, _u32, _u32, _vp, _vp]
    L.orc_nw_draw.restype = ctypes.c_int
    L.orc_mm.argtypes = [_i64, _i32, _i32, _vp, _vp, _vp]
    L.orc_mm.restype = _i64
    L.orc_update_side_w.argtypes = [_i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _d, _u64,
                                    _u32, _u32, _vp, _i32]
    L.orc_update_side_w.restype = _i64
    L.orc_tau_cols.argtypes = [_i64, _vp, _vp, _d, _d, _u64, _u32, _u32, _vp]
    L.orc_tau_cols.restype = None
    L.orc_lmeans.argtypes = [_i64, _i32, _i32, _vp, _d, _i32, _i32, _vp, _vp]
    L.orc_lmeans.restype = _i64
    L.orc_mm_sel.argtypes = [_i64, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.orc_mm_sel.restype = _i64
    _lib = L
    return L


def ptr(a):
    """Raw data pointer of a C-contiguous numpy array (None: a null pointer)."""
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


# --- thin numpy-facing wrappers ---------------------------------------------

def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(ptr(c), ptr(k), ptr(o))
    return o


def philox_batch(ctr, seed):
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    o = np.zeros_like(c)
    lib().orc_philox_batch(c.shape[0], ptr(c), np.uint64(seed), ptr(o))
    return o


def normals(seed, c0, c1, c2, n):
    z = np.zeros(max(n, 1), dtype=np.float64)
    lib().orc_normals(seed, c0, c1, c2, n, ptr(z))
    return z[:n]


def gamma(seed, c0, c1, c2, shape):
    return lib().orc_gamma(seed, c0, c1, c2, shape)


def cholesky(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    L = np.zeros_like(A)
    rc = lib().orc_cholesky(A.shape[0], ptr(A), ptr(L))
    return L if rc == 0 else None


def seq_mean(val):
    v = np.ascontiguousarray(val, dtype=np.float32)
    return lib().orc_seq_mean(v.size, ptr(v))
