"""Python binding of libkl (ctypes over the C ABI in ``include/kl.h``).

Argument marshalling only: every step of the stencil path runs in the HIP
kernels of ``libkl.so``.  PyTorch provides device memory and streams.  The
functions keep the C names; tensors are passed as device pointers, ``stream``
defaults to torch's current stream.  A missing or unloadable ``libkl.so``
raises at import: there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import (POINTER, Structure, byref, c_char_p, c_double, c_int, c_int32, c_int64,
                    c_size_t, c_uint32, c_uint64, c_void_p)

import numpy as np
import torch  # noqa: F401  (loads torch's HIP runtime before libkl binds to it)

from . import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
# KL_LIBRARY may name another build of this same library (the tests use it
# for a build whose host code carries the address and undefined-behaviour
# sanitizers); there is no fallback when the named file is missing.
LIB_PATH = os.environ.get("KL_LIBRARY") or os.path.join(HERE, "libkl.so")

F32, F64 = 0, 1
BC_ZWALL_ZEROGRAD, BC_ZWALL_NOPEN, BC_ZPERIODIC = 0, 1, 2
ADVEC_U, DIFF_UVW, STEP, ADVEC_U_2I5, DIFF_SMAG, ADVEC_DIFF = 0, 1, 2, 3, 4, 5
TUNE_ADVEC_U, TUNE_DIFF_UVW, TUNE_STEP, TUNE_PAIR, TUNE_ADVEC_U_2I5, TUNE_DIFF_SMAG, TUNE_ADVEC_DIFF = \
    1, 2, 4, 8, 16, 32, 64
BATCH_ZERO_TENDENCIES, BATCH_FILL_GHOSTS, BATCH_SUMS = 1, 2, 4
KERNEL_NAMES = {ADVEC_U: "advec_u", DIFF_UVW: "diff_uvw", STEP: "step", ADVEC_U_2I5: "advec_u_2i5",
                DIFF_SMAG: "diff_smag", ADVEC_DIFF: "advec_diff"}
OK, ERR_INVALID, ERR_DEVICE, ERR_NOMEM, ERR_BUDGET, ERR_AGAIN, ERR_NOTFOUND, ERR_IO = 0, -1, -2, -3, -4, -5, -6, -7

TORCH_DTYPE = {F32: torch.float32, F64: torch.float64}
NP_DTYPE = {F32: np.float32, F64: np.float64}


class kl_grid_t(Structure):
    _fields_ = [("itot", c_int32), ("jtot", c_int32), ("ktot", c_int32), ("gc", c_int32),
                ("off", c_int64), ("jstride", c_int64), ("kstride", c_int64),
                ("dxi", c_double), ("dyi", c_double), ("dzi", c_void_p), ("dzhi", c_void_p),
                ("dtype", c_int32), ("bc", c_int32)]


class kl_request_t(Structure):
    _fields_ = [("itot", c_int32), ("jtot", c_int32), ("ktot", c_int32), ("dtype", c_int32),
                ("bc", c_int32), ("nsteps", c_int32), ("dt", c_double), ("visc", c_double),
                ("seed", c_uint64)]


class kl_result_t(Structure):
    _fields_ = [("state", c_int32), ("err", c_int32), ("t_arrive_ns", c_int64),
                ("t_admit_ns", c_int64), ("t_done_ns", c_int64), ("checksum", c_double * 9),
                ("fields", c_void_p * 3), ("off", c_int64), ("jstride", c_int64), ("kstride", c_int64)]


class KLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libkl error {code}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                      "python paper_2303_12374_amd/build.py")
_lib = ctypes.CDLL(LIB_PATH)

_G = POINTER(kl_grid_t)
_sig = {
    "kl_version": (c_char_p, []),
    "kl_last_error": (c_char_p, []),
    "kl_layout": (c_int, [c_int32, c_int32, c_int32, c_int32, POINTER(c_int64), POINTER(c_int64),
                          POINTER(c_int64), POINTER(c_int64)]),
    "kl_layout_gc": (c_int, [c_int32, c_int32, c_int32, c_int32, c_int32, POINTER(c_int64), POINTER(c_int64),
                             POINTER(c_int64), POINTER(c_int64)]),
    "kl_fill_ghosts": (c_int, [_G, c_void_p, c_void_p, c_void_p, c_void_p]),
    "kl_fill_scalar": (c_int, [_G, c_void_p, c_void_p]),
    "kl_advec_u_2i5": (c_int, [_G, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "kl_diff_smag": (c_int, [_G, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p]),
    "kl_advec_u": (c_int, [_G, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "kl_diff_uvw": (c_int, [_G, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                            c_double, c_void_p]),
    "kl_advec_diff": (c_int, [_G, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_double, c_void_p]),
    "kl_euler": (c_int, [_G, c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                         c_void_p]),
    "kl_step": (c_int, [_G, c_double, c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                        c_void_p, c_void_p]),
    "kl_step_fused": (c_int, [_G, c_double, c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p]),
    "kl_reduce_fp64": (c_int, [_G, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "kl_reduce_fp64_noalloc": (c_int, [_G, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "kl_generate_fields": (c_int, [_G, c_uint64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "kl_hash_interior": (c_int, [_G, c_void_p, c_void_p, c_void_p]),
    "kl_stream_probe": (c_int, [c_int32, c_int32, POINTER(c_void_p), POINTER(c_void_p), c_int64, c_int32,
                                c_void_p]),
    "kl_num_variants": (c_int, [c_int32, c_int32]),
    "kl_variant_name": (c_int, [c_int32, c_int32, c_int32, c_char_p, c_size_t]),
    "kl_variant_eligible": (c_int, [_G, c_int32, c_int32, POINTER(c_void_p)]),
    "kl_launch_variant": (c_int, [_G, c_int32, c_int32, POINTER(c_void_p), c_double, c_void_p]),
    "kl_launch_variant_dt": (c_int, [_G, c_int32, c_int32, POINTER(c_void_p), c_double, c_double, c_void_p]),
    "kl_selected_variant": (c_int, [_G, c_int32]),
    "kl_set_wisdom_dir": (c_int, [c_char_p]),
    "kl_clear_plan_cache": (c_int, []),
    "kl_wisdom_lookup": (c_int, [c_char_p, c_int32, c_int32, c_char_p, c_char_p, c_int32, c_int32, c_int32,
                                 c_int32, c_char_p, c_size_t, POINTER(c_int32)]),
    "kl_tune": (c_int, [_G, POINTER(c_void_p), c_uint32, c_char_p, c_double, c_void_p,
                        POINTER(c_double), c_int32, POINTER(c_int32)]),
    "kl_set_capture": (c_int, [c_char_p, c_char_p]),
    "kl_capture": (c_int, [_G, c_int32, POINTER(c_void_p), c_double, c_double, c_char_p, c_void_p]),
    "kl_capture_info": (c_int, [c_char_p, c_char_p, c_size_t]),
    "kl_tune_capture": (c_int, [c_char_p, c_char_p, c_double, c_void_p, POINTER(c_double), c_int32,
                                POINTER(c_int32)]),
    "kl_batch_create": (c_int, [_G, POINTER(c_void_p), c_int32, c_double, c_int32, c_void_p,
                                POINTER(c_void_p)]),
    "kl_batch_create_ex": (c_int, [_G, POINTER(c_void_p), c_int32, c_double, c_uint32, c_void_p, c_void_p,
                                   POINTER(c_void_p)]),
    "kl_batch_tune": (c_int, [c_void_p, c_char_p, c_double, c_void_p, c_void_p, c_int32, POINTER(c_int32)]),
    "kl_batch_group": (c_int, [c_void_p, c_int32, POINTER(c_int32), c_char_p, c_size_t, POINTER(c_int64)]),
    "kl_batch_run": (c_int, [c_void_p, c_void_p]),
    "kl_batch_info": (c_int, [c_void_p, POINTER(c_int32), POINTER(c_int64)]),
    "kl_batch_destroy": (c_int, [c_void_p]),
    "kl_server_create": (c_int, [c_void_p, c_size_t, c_size_t, POINTER(c_void_p)]),
    "kl_submit": (c_int, [c_void_p, POINTER(kl_request_t), POINTER(c_uint64)]),
    "kl_poll": (c_int, [c_void_p, c_uint64, POINTER(kl_result_t)]),
    "kl_release": (c_int, [c_void_p, c_uint64]),
    "kl_server_stats": (c_int, [c_void_p, POINTER(c_int64)]),
    "kl_server_destroy": (c_int, [c_void_p]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

DECLARED = tuple(_sig)


def _check(rc):
    if rc < 0:
        raise KLError(rc, _lib.kl_last_error().decode())
    return rc


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.data_ptr()
    return int(x)


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _fields6(fields):
    """C array of the field pointers (6, or 7 with the eddy viscosity)."""
    ptrs = [_ptr(f) for f in fields]
    ptrs += [None] * (max(6, len(ptrs)) - len(ptrs))
    return (c_void_p * len(ptrs))(*ptrs)


# ---------------------------------------------------------------------------
# thin wrappers with the C names
# ---------------------------------------------------------------------------

def kl_version() -> str:
    return _lib.kl_version().decode()


def kl_last_error() -> str:
    return _lib.kl_last_error().decode()


def kl_layout(itot, jtot, ktot, dtype):
    off, js, ks, alloc = c_int64(), c_int64(), c_int64(), c_int64()
    _check(_lib.kl_layout(itot, jtot, ktot, dtype, byref(off), byref(js), byref(ks), byref(alloc)))
    return off.value, js.value, ks.value, alloc.value


def kl_layout_gc(itot, jtot, ktot, dtype, gc):
    off, js, ks, alloc = c_int64(), c_int64(), c_int64(), c_int64()
    _check(_lib.kl_layout_gc(itot, jtot, ktot, dtype, gc, byref(off), byref(js), byref(ks), byref(alloc)))
    return off.value, js.value, ks.value, alloc.value


def kl_fill_ghosts(g, u, v, w, stream=None):
    _check(_lib.kl_fill_ghosts(byref(_cg(g)), _ptr(u), _ptr(v), _ptr(w), _stream(stream)))


def kl_fill_scalar(g, f, stream=None):
    _check(_lib.kl_fill_scalar(byref(_cg(g)), _ptr(f), _stream(stream)))


def kl_advec_u_2i5(g, ut, u, v, w, stream=None):
    _check(_lib.kl_advec_u_2i5(byref(_cg(g)), _ptr(ut), _ptr(u), _ptr(v), _ptr(w), _stream(stream)))


def kl_diff_smag(g, ut, vt, wt, u, v, w, evisc, stream=None):
    _check(_lib.kl_diff_smag(byref(_cg(g)), _ptr(ut), _ptr(vt), _ptr(wt), _ptr(u), _ptr(v), _ptr(w),
                             _ptr(evisc), _stream(stream)))


def kl_advec_u(g, ut, u, v, w, stream=None):
    _check(_lib.kl_advec_u(byref(_cg(g)), _ptr(ut), _ptr(u), _ptr(v), _ptr(w), _stream(stream)))


def kl_diff_uvw(g, ut, vt, wt, u, v, w, visc, stream=None):
    _check(_lib.kl_diff_uvw(byref(_cg(g)), _ptr(ut), _ptr(vt), _ptr(wt), _ptr(u), _ptr(v), _ptr(w),
                            float(visc), _stream(stream)))


def kl_advec_diff(g, ut, vt, wt, u, v, w, visc, stream=None):
    _check(_lib.kl_advec_diff(byref(_cg(g)), _ptr(ut), _ptr(vt), _ptr(wt), _ptr(u), _ptr(v), _ptr(w),
                              float(visc), _stream(stream)))


def kl_euler(g, dt, u, v, w, ut, vt, wt, stream=None):
    _check(_lib.kl_euler(byref(_cg(g)), float(dt), _ptr(u), _ptr(v), _ptr(w), _ptr(ut), _ptr(vt),
                         _ptr(wt), _stream(stream)))


def kl_step(g, visc, dt, u, v, w, ut, vt, wt, stream=None):
    _check(_lib.kl_step(byref(_cg(g)), float(visc), float(dt), _ptr(u), _ptr(v), _ptr(w), _ptr(ut),
                        _ptr(vt), _ptr(wt), _stream(stream)))


def kl_step_fused(g, visc, dt, u, v, w, u_out, v_out, w_out, stream=None):
    _check(_lib.kl_step_fused(byref(_cg(g)), float(visc), float(dt), _ptr(u), _ptr(v), _ptr(w), _ptr(u_out),
                              _ptr(v_out), _ptr(w_out), _stream(stream)))


def kl_reduce_fp64(g, what, f0, f1, f2, out, stream=None):
    _check(_lib.kl_reduce_fp64(byref(_cg(g)), what, _ptr(f0), _ptr(f1), _ptr(f2), _ptr(out),
                               _stream(stream)))


def kl_reduce_fp64_noalloc(g, what, f0, f1, f2, out, stream=None):
    _check(_lib.kl_reduce_fp64_noalloc(byref(_cg(g)), what, _ptr(f0), _ptr(f1), _ptr(f2), _ptr(out),
                                       _stream(stream)))


def kl_generate_fields(g, seed, u, v, w, stream=None):
    _check(_lib.kl_generate_fields(byref(_cg(g)), c_uint64(seed), _ptr(u), _ptr(v), _ptr(w),
                                   _stream(stream)))


def kl_hash_interior(g, f, out, stream=None):
    _check(_lib.kl_hash_interior(byref(_cg(g)), _ptr(f), _ptr(out), _stream(stream)))


def kl_stream_probe(srcs, dsts, nbytes, nontemporal=False, stream=None):
    src = (c_void_p * len(srcs))(*[_ptr(x) for x in srcs])
    dst = (c_void_p * len(dsts))(*[_ptr(x) for x in dsts])
    _check(_lib.kl_stream_probe(len(srcs), len(dsts), src, dst, int(nbytes), int(bool(nontemporal)),
                                _stream(stream)))


def kl_num_variants(kernel, dtype) -> int:
    return _check(_lib.kl_num_variants(kernel, dtype))


def kl_variant_name(kernel, dtype, index) -> str:
    buf = ctypes.create_string_buffer(128)
    _check(_lib.kl_variant_name(kernel, dtype, index, buf, 128))
    return buf.value.decode()


def kl_variant_eligible(g, kernel, index, fields) -> bool:
    return bool(_check(_lib.kl_variant_eligible(byref(_cg(g)), kernel, index, _fields6(fields))))


def kl_launch_variant(g, kernel, index, fields, visc=0.0, stream=None):
    _check(_lib.kl_launch_variant(byref(_cg(g)), kernel, index, _fields6(fields), float(visc),
                                  _stream(stream)))


def kl_launch_variant_dt(g, kernel, index, fields, visc=0.0, dt=0.0, stream=None):
    _check(_lib.kl_launch_variant_dt(byref(_cg(g)), kernel, index, _fields6(fields), float(visc), float(dt),
                                     _stream(stream)))


def kl_selected_variant(g, kernel) -> int:
    return _check(_lib.kl_selected_variant(byref(_cg(g)), kernel))


def kl_set_wisdom_dir(path):
    _check(_lib.kl_set_wisdom_dir(None if path is None else str(path).encode()))


def kl_clear_plan_cache():
    _check(_lib.kl_clear_plan_cache())


def kl_wisdom_lookup(wisdom_dir, kernel, dtype, device_name, arch, itot, jtot, ktot, cu_count=0):
    buf = ctypes.create_string_buffer(128)
    level = c_int32()
    _check(_lib.kl_wisdom_lookup(None if wisdom_dir is None else str(wisdom_dir).encode(), kernel, dtype,
                                 device_name.encode(), arch.encode(), cu_count, itot, jtot, ktot, buf, 128,
                                 byref(level)))
    return buf.value.decode(), level.value


def kl_tune(g, fields, kernel_mask, wisdom_dir=None, budget_s=60.0, stream=None, max_timings=512):
    out = (c_double * (2 * max_timings))()
    n = c_int32()
    _check(_lib.kl_tune(byref(_cg(g)), _fields6(fields), kernel_mask,
                        None if wisdom_dir is None else str(wisdom_dir).encode(), float(budget_s),
                        _stream(stream), out, max_timings, byref(n)))
    return [(int(out[2 * i]), out[2 * i + 1]) for i in range(n.value)]


def kl_set_capture(kernels, directory=None):
    """kernels: comma-separated kernel names, or None / "" to stop capturing."""
    _check(_lib.kl_set_capture(None if not kernels else kernels.encode(),
                               None if directory is None else str(directory).encode()))


def kl_capture(g, kernel, fields, visc, dt, path, stream=None):
    _check(_lib.kl_capture(byref(_cg(g)), kernel, _fields6(fields), float(visc), float(dt), str(path).encode(),
                           _stream(stream)))


def kl_capture_info(path) -> dict:
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(_lib.kl_capture_info(str(path).encode(), buf, 1 << 16))
    return json.loads(buf.value.decode())


def kl_tune_capture(path, wisdom_dir=None, budget_s=60.0, stream=None, max_timings=512):
    out = (c_double * (2 * max_timings))()
    n = c_int32()
    _check(_lib.kl_tune_capture(str(path).encode(), None if wisdom_dir is None else str(wisdom_dir).encode(),
                                float(budget_s), _stream(stream), out, max_timings, byref(n)))
    return [(int(out[2 * i]), out[2 * i + 1]) for i in range(n.value)]


def read_capture(path):
    """(header dict, {array name: numpy array}) of a capture file, read on the host."""
    import json
    with open(path, "rb") as f:
        magic = f.readline()
        if magic != b"KLCAP 1\n":
            raise ValueError(f"{path} is not a KLCAP 1 file")
        hdr = json.loads(f.readline().decode())
        dt = np.float32 if hdr["dtype"] == "f32" else np.float64
        arrays = {a["name"]: np.fromfile(f, dtype=dt, count=int(a["elems"])) for a in hdr["arrays"]}
    return hdr, arrays


def kl_batch_create(grids, fields, visc, zero_tendencies=True, stream=None):
    n = len(grids)
    arr = (kl_grid_t * n)(*[_cg(g) for g in grids])
    flat = (c_void_p * (6 * n))(*[_ptr(f) for fs in fields for f in fs])
    h = c_void_p()
    _check(_lib.kl_batch_create(arr, flat, n, float(visc), int(bool(zero_tendencies)), _stream(stream),
                                byref(h)))
    return h.value


def kl_batch_create_ex(grids, fields, visc, flags, sums=None, stream=None):
    """kl_batch_create with the graph's other steps (BATCH_* flags); sums: a
    float64 device tensor of 3 * len(grids) values for BATCH_SUMS."""
    n = len(grids)
    arr = (kl_grid_t * n)(*[_cg(g) for g in grids])
    flat = (c_void_p * (6 * n))(*[_ptr(f) for fs in fields for f in fs])
    h = c_void_p()
    _check(_lib.kl_batch_create_ex(arr, flat, n, float(visc), int(flags), _ptr(sums),
                                   _stream(stream), byref(h)))
    return h.value


def kl_batch_run(batch, stream=None):
    _check(_lib.kl_batch_run(c_void_p(batch), _stream(stream)))


def kl_batch_info(batch):
    nk, nt = c_int32(), c_int64()
    _check(_lib.kl_batch_info(c_void_p(batch), byref(nk), byref(nt)))
    return nk.value, nt.value


def kl_batch_tune(batch, wisdom_dir=None, budget_s=60.0, stream=None, max_timings=256):
    """Tune a batch as a whole; returns [(configuration index or -1 for the
    per-grid selection, ms or -1)]."""
    out = (c_double * (2 * max_timings))()
    n = c_int32()
    _check(_lib.kl_batch_tune(c_void_p(batch), None if wisdom_dir is None else str(wisdom_dir).encode(),
                              float(budget_s), _stream(stream), out, max_timings, byref(n)))
    return [(int(out[2 * i]), out[2 * i + 1]) for i in range(n.value)]


def kl_batch_groups(batch):
    """[(dtype, configuration name, tiles)] of the batch's persistent kernels."""
    res = []
    g = 0
    while True:
        dt = c_int32()
        nt = c_int64()
        buf = ctypes.create_string_buffer(128)
        rc = _lib.kl_batch_group(c_void_p(batch), g, byref(dt), buf, 128, byref(nt))
        if rc == ERR_NOTFOUND:
            return res
        _check(rc)
        res.append((dt.value, buf.value.decode(), nt.value))
        g += 1


def kl_batch_destroy(batch):
    _check(_lib.kl_batch_destroy(c_void_p(batch)))


def kl_server_create(arena, arena_bytes, budget_bytes):
    h = c_void_p()
    _check(_lib.kl_server_create(_ptr(arena), int(arena_bytes), int(budget_bytes), byref(h)))
    return h.value


def kl_submit(srv, itot, jtot, ktot, dtype, bc, nsteps, dt, visc, seed):
    req = kl_request_t(itot, jtot, ktot, dtype, bc, nsteps, dt, visc, seed)
    t = c_uint64()
    _check(_lib.kl_submit(c_void_p(srv), byref(req), byref(t)))
    return t.value


def kl_poll(srv, ticket):
    """Returns (rc, kl_result_t); rc is OK or ERR_AGAIN."""
    res = kl_result_t()
    rc = _lib.kl_poll(c_void_p(srv), c_uint64(ticket), byref(res))
    if rc not in (OK, ERR_AGAIN):
        _check(rc)
    return rc, res


def kl_release(srv, ticket):
    _check(_lib.kl_release(c_void_p(srv), c_uint64(ticket)))


def kl_server_stats(srv):
    out = (c_int64 * 5)()
    _check(_lib.kl_server_stats(c_void_p(srv), out))
    return list(out)


def kl_server_destroy(srv):
    _check(_lib.kl_server_destroy(c_void_p(srv)))


# ---------------------------------------------------------------------------
# Grid: device metrics + the kl_grid_t descriptor
# ---------------------------------------------------------------------------

def _cg(g):
    return g.c if isinstance(g, Grid) else g


class Grid:
    """A grid with device metrics.  ``dtype`` is F32 or F64.

    The vertical grid is the centers-primary tanh stretch of
    :func:`inputs.zgrid` (uniform when ``bc == BC_ZPERIODIC`` or
    ``gamma == 0``); ``dx = 1/itot``, ``dy = 1/jtot``.  ``gc`` ghost cells per
    side in x and y (1, or 3 for advec_u_2i5).  ``layout`` defaults to
    :func:`kl_layout_gc`.
    """

    def __init__(self, itot, jtot, ktot, dtype=F32, bc=BC_ZWALL_ZEROGRAD, gamma=1.5, layout=None,
                 device="cuda", gc=1):
        self.itot, self.jtot, self.ktot, self.dtype, self.bc = itot, jtot, ktot, dtype, bc
        self.gc = gc
        self.device = torch.device(device)
        if layout is None:
            layout = kl_layout_gc(itot, jtot, ktot, dtype, gc)
        self.off, self.js, self.ks, self.alloc = (int(x) for x in layout)
        Lz = inputs.domain_height(itot, jtot, ktot)
        self.zg = inputs.zgrid(ktot, Lz, 0.0 if bc == BC_ZPERIODIC else gamma)
        npd = NP_DTYPE[dtype]
        # metrics in the field dtype (the FP32 path rounds them once, here)
        self.dzi_h = self.zg["dzi"].astype(npd)
        self.dzhi_h = self.zg["dzhi"].astype(npd)
        self.dxi = float(npd(itot))
        self.dyi = float(npd(jtot))
        self.dzi = torch.from_numpy(self.dzi_h.copy()).to(self.device)
        self.dzhi = torch.from_numpy(self.dzhi_h.copy()).to(self.device)
        self.c = kl_grid_t(itot, jtot, ktot, gc, self.off, self.js, self.ks, self.dxi, self.dyi,
                           self.dzi.data_ptr(), self.dzhi.data_ptr(), dtype, bc)

    @property
    def tdtype(self):
        return TORCH_DTYPE[self.dtype]

    @property
    def npoints(self):
        return self.itot * self.jtot * self.ktot

    def full(self, value=math.nan):
        return torch.full((self.alloc,), value, dtype=self.tdtype, device=self.device)

    def box(self, t):
        """(ktot+2, jtot+2*gc, itot+2*gc) strided view of a flat field tensor;
        box[k, j, i] is element (i+1-gc, j+1-gc, k)."""
        g = self.gc
        return t.as_strided((self.ktot + 2, self.jtot + 2 * g, self.itot + 2 * g), (self.ks, self.js, 1),
                            t.storage_offset() + self.off - (g - 1) * (self.js + 1))

    def interior(self, t):
        g = self.gc
        return self.box(t)[1:self.ktot + 1, g:self.jtot + g, g:self.itot + g]

    def upload(self, interior_np, fill=math.nan):
        """Device field holding ``interior_np`` (rounded to the dtype); ghosts = fill."""
        t = self.full(fill)
        self.interior(t).copy_(torch.from_numpy(np.ascontiguousarray(interior_np, dtype=NP_DTYPE[self.dtype])))
        return t

    def zeros_interior(self, fill=math.nan):
        t = self.full(fill)
        self.interior(t).zero_()
        return t
