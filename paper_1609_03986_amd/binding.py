"""Thin Python binding over the C ABI of liblatch.so (include/latch.h).

Argument marshalling only: every step of extraction and matching runs in the
library's HIP kernels.  torch is used for device memory and streams.  The
binding fails loudly if the library has not been built; there is no CPU
fallback.

The functions keep the C names:
    latch_create(triplets) -> handle
    latch_destroy(handle)
    latch_extract(handle, img, kps, desc=None, stream=None) -> desc
    hamming_knn(handle, query, train, k=2, ratio=0.8, path="auto", ...) -> (idx, dist, accept)
    hamming_knn_workspace_size(handle, nq, nt, path) -> bytes; latch_reserve(handle, bytes)
    latch_check_errors(handle, stream=None, clear=True) -> flags
    latch_rotation_table() -> (cos_q14, sin_q14)   (host only)
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblatch.so")

LATCH_OK, LATCH_EINVAL, LATCH_ENOMEM, LATCH_EDEVICE, LATCH_ERANGE, LATCH_EWORKSPACE = 0, -1, -2, -3, -4, -5
PATHS = {"auto": 0, "mfma": 1, "popcount": 2, "fp4": 3}
FLAG_BAD_KEYPOINT = 1
FLAG_BAD_IMAGE = 2
FLAG_BAD_PAIR = 4
NO_NEIGHBOUR_DIST = 513
STATUS_NAMES = {0: "LATCH_OK", -1: "LATCH_EINVAL", -2: "LATCH_ENOMEM", -3: "LATCH_EDEVICE",
                -4: "LATCH_ERANGE", -5: "LATCH_EWORKSPACE"}

# Every symbol include/latch.h declares.
EXPORTS = ("latch_create", "latch_create_geometry", "latch_destroy", "hamming_knn_workspace_size",
           "hamming_knn_batch_workspace_size", "latch_detect_workspace_size",
           "latch_extract_batch_workspace_size", "latch_reserve",
           "latch_extract", "latch_extract_batch",
           "latch_extract_dense", "hamming_knn_window", "latch_detect",
           "hamming_knn", "hamming_knn_noalloc",
           "hamming_knn_batch", "latch_plan_create", "latch_plan_run", "latch_plan_destroy",
           "latch_get_tuning", "latch_set_tuning",
           "latch_check_errors",
           "latch_last_error", "latch_rotation_table", "latch_version", "latch_timing_enable",
           "latch_timing_read")
KERNELS = ("extract", "dense_extract", "knn_window", "detect", "knn_mfma", "knn_fp4", "knn_popcount", "knn_merge", "knn_batch_mfma",
           "knn_batch_popcount")


class LatchError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


_lib = None


def load_library():
    """Load liblatch.so (built in-tree by paper_1609_03986_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblatch.so is not built; run `python -m paper_1609_03986_amd.build`")
    # torch ships its own libamdhip64 with the same soname as the system one.
    # Loading torch first makes the dynamic linker bind liblatch.so to that
    # runtime; loading liblatch.so first would put two HIP runtimes in the
    # process, and the second one to initialise finds no GPU.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, F = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float
    lib.latch_create.argtypes = [ctypes.POINTER(P), P]
    lib.latch_create.restype = I
    lib.latch_create_geometry.argtypes = [ctypes.POINTER(P), P, I, I, P]
    lib.latch_create_geometry.restype = I
    lib.latch_destroy.argtypes = [P]
    lib.latch_destroy.restype = None
    SZ = ctypes.POINTER(ctypes.c_size_t)
    lib.hamming_knn_workspace_size.argtypes = [P, I64, I64, I, SZ]
    lib.hamming_knn_workspace_size.restype = I
    lib.hamming_knn_batch_workspace_size.argtypes = [P, I, I64, SZ]
    lib.hamming_knn_batch_workspace_size.restype = I
    lib.latch_detect_workspace_size.argtypes = [P, I, I, SZ]
    lib.latch_detect_workspace_size.restype = I
    lib.latch_extract_batch_workspace_size.argtypes = [P, I, I64, SZ]
    lib.latch_extract_batch_workspace_size.restype = I
    lib.latch_reserve.argtypes = [P, ctypes.c_size_t, SZ]
    lib.latch_reserve.restype = I
    lib.latch_extract.argtypes = [P, P, I, I, I, P, I64, P, P]
    lib.latch_extract.restype = I
    lib.latch_extract_batch.argtypes = [P, P, I, P, P, I64, P, P, P]
    lib.latch_extract_batch.restype = I
    lib.latch_extract_dense.argtypes = [P, P, I, I, I, I, I, I, I, P, P]
    lib.latch_extract_dense.restype = I
    lib.hamming_knn_window.argtypes = [P, P, P, I, I, I, I, F, P, P, P, P]
    lib.hamming_knn_window.restype = I
    lib.latch_detect.argtypes = [P, P, I, I, I, I, P, I64, P, P, I, P]
    lib.latch_detect.restype = I
    lib.hamming_knn.argtypes = [P, P, I64, P, I64, I, F, P, P, P, I, P]
    lib.hamming_knn_noalloc.argtypes = [P, P, I64, P, I64, I, F, P, P, P, I, P]
    lib.hamming_knn_noalloc.restype = I
    lib.hamming_knn_batch.argtypes = [P, P, I64, P, I64, P, I, I, F, P, P, P, I64, I, P]
    lib.hamming_knn_batch.restype = I
    lib.latch_plan_create.argtypes = [P, P, ctypes.POINTER(P)]
    lib.latch_plan_create.restype = I
    lib.latch_plan_run.argtypes = [P, P]
    lib.latch_plan_run.restype = I
    lib.latch_plan_destroy.argtypes = [P]
    lib.latch_plan_destroy.restype = None
    lib.latch_get_tuning.argtypes = [P, P]
    lib.latch_get_tuning.restype = I
    lib.latch_set_tuning.argtypes = [P, P]
    lib.latch_set_tuning.restype = I
    lib.hamming_knn.restype = I
    lib.latch_check_errors.argtypes = [P, P, ctypes.POINTER(ctypes.c_uint32), I]
    lib.latch_check_errors.restype = I
    lib.latch_last_error.argtypes = [P]
    lib.latch_last_error.restype = ctypes.c_char_p
    lib.latch_rotation_table.argtypes = [P, P]
    lib.latch_rotation_table.restype = I
    lib.latch_timing_enable.argtypes = [P, I]
    lib.latch_timing_enable.restype = I
    lib.latch_timing_read.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(I),
                                      ctypes.POINTER(ctypes.c_double)]
    lib.latch_timing_read.restype = I
    lib.latch_version.argtypes = []
    lib.latch_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(h, rc):
    if rc != LATCH_OK:
        msg = load_library().latch_last_error(h)
        raise LatchError(rc, msg.decode() if msg else "")


def _with_workspace(h, call, size):
    """Run `call()`; if the handle's workspace is too small (the call then
    enqueued nothing), reserve what `size()` reports and run it again.  The
    reserve is the explicit set-up call of the C ABI (it waits for the device
    only when it replaces a smaller workspace)."""
    rc = call()
    if rc == LATCH_EWORKSPACE:
        latch_reserve(h, size())
        rc = call()
    _check(h, rc)


def _size_out(h, fn, *args):
    out = ctypes.c_size_t()
    _check(h, fn(h, *args, ctypes.byref(out)))
    return out.value


def hamming_knn_workspace_size(h, nq, nt, path="auto"):
    """Workspace bytes hamming_knn needs for these sizes on this handle."""
    return _size_out(h, load_library().hamming_knn_workspace_size, int(nq), int(nt), PATHS[path])


def hamming_knn_batch_workspace_size(h, n_pairs, out_rows):
    return _size_out(h, load_library().hamming_knn_batch_workspace_size, int(n_pairs), int(out_rows))


def latch_detect_workspace_size(h, height, width):
    return _size_out(h, load_library().latch_detect_workspace_size, int(height), int(width))


def latch_extract_batch_workspace_size(h, n_images, max_kps):
    """Workspace bytes of a batched extraction's spatial order (0 if none)."""
    return _size_out(h, load_library().latch_extract_batch_workspace_size, int(n_images),
                     int(max_kps))


def latch_reserve(h, nbytes=0):
    """Make the handle's workspace at least nbytes; returns the bytes it holds."""
    held = ctypes.c_size_t()
    _check(h, load_library().latch_reserve(h, int(nbytes), ctypes.byref(held)))
    return held.value


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous() and not (name == "img" and t.stride(1) == 1):
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def latch_rotation_table():
    """Host-only rotation table of the resampling rule: (cos_q14, sin_q14) int16[4096]."""
    c = np.zeros(4096, np.int16)
    s = np.zeros(4096, np.int16)
    rc = load_library().latch_rotation_table(c.ctypes.data_as(ctypes.c_void_p),
                                             s.ctypes.data_as(ctypes.c_void_p))
    _check(None, rc)
    return c, s


def latch_version():
    return load_library().latch_version().decode()


def latch_create(triplets):
    """Create a handle on the current device from uint8[512, 3, 2] triplets (host)."""
    trip = np.ascontiguousarray(np.asarray(triplets, np.uint8).reshape(512, 3, 2))
    h = ctypes.c_void_p()
    rc = load_library().latch_create(ctypes.byref(h), trip.ctypes.data_as(ctypes.c_void_p))
    if rc != LATCH_OK:
        raise LatchError(rc, "latch_create failed")
    return h


def latch_create_geometry(triplets, window=64, patch=8, weights=None):
    """Create a handle with window side `window` (48, 64), patch side `patch`
    (7, 8) and integer weights uint8[patch, patch] in [0, 128] (None: ones)."""
    trip = np.ascontiguousarray(np.asarray(triplets, np.uint8).reshape(512, 3, 2))
    wp = None
    if weights is not None:
        w = np.ascontiguousarray(np.asarray(weights, np.uint8).reshape(patch, patch))
        wp = w.ctypes.data_as(ctypes.c_void_p)
    h = ctypes.c_void_p()
    rc = load_library().latch_create_geometry(ctypes.byref(h), trip.ctypes.data_as(ctypes.c_void_p),
                                              int(window), int(patch), wp)
    if rc != LATCH_OK:
        raise LatchError(rc, "latch_create_geometry failed")
    return h


def latch_destroy(h):
    load_library().latch_destroy(h)


def latch_extract(h, img, kps, desc=None, stream=None):
    """Extract descriptors; returns desc, torch.int32 [n, 16] holding the uint32 words.

    img: uint8 [H, W] CUDA tensor; a row stride larger than W is passed as the pitch.
    kps: float32 [n, 4] CUDA tensor of (x, y, angle_deg, scale).
    """
    import torch
    if img.dim() != 2:
        raise ValueError("img must be 2-D")
    if kps.dim() != 2 or kps.shape[1] != 4:
        raise ValueError("kps must be [n, 4]")
    n = kps.shape[0]
    if desc is None:
        desc = torch.empty((n, 16), dtype=torch.int32, device=kps.device)
    elif tuple(desc.shape) != (n, 16):
        raise ValueError("desc must be [n, 16]")
    H, W = img.shape
    rc = load_library().latch_extract(h, _dev(img, torch.uint8, "img"), H, W, img.stride(0),
                                      _dev(kps, torch.float32, "kps"), n,
                                      _dev(desc, torch.int32, "desc"), _stream_ptr(stream))
    _check(h, rc)
    return desc


def latch_extract_dense(h, img, x0, y0, gw, gh, desc=None, stream=None):
    """Descriptors of every pixel of [x0, x0 + gw) x [y0, y0 + gh), upright at
    scale 1: int32 [gh * gw, 16] (uint32 words), raster order."""
    import torch
    if img.dim() != 2:
        raise ValueError("img must be 2-D")
    if desc is None:
        desc = torch.empty((gh * gw, 16), dtype=torch.int32, device=img.device)
    H, W = img.shape
    rc = load_library().latch_extract_dense(h, _dev(img, torch.uint8, "img"), H, W, img.stride(0),
                                            int(x0), int(y0), int(gw), int(gh),
                                            _dev(desc, torch.int32, "desc"), _stream_ptr(stream))
    _check(h, rc)
    return desc


def hamming_knn_window(h, query, train, gw, gh, radius, k=2, ratio=0.8, stream=None):
    """Dense matching of two gh x gw descriptor grids within +/- radius:
    (idx int32 [n, k] raster indices, dist int32 [n, k], accept uint8 [n])."""
    import torch
    n = gh * gw
    dev = query.device
    idx = torch.empty((n, k), dtype=torch.int32, device=dev)
    dist = torch.empty((n, k), dtype=torch.int32, device=dev)
    acc = torch.empty((n,), dtype=torch.uint8, device=dev)
    rc = load_library().hamming_knn_window(h, _dev(query, torch.int32, "query"),
                                           _dev(train, torch.int32, "train"), int(gw), int(gh),
                                           int(radius), int(k), float(ratio),
                                           _dev(idx, torch.int32, "idx"), _dev(dist, torch.int32, "dist"),
                                           _dev(acc, torch.uint8, "accept"), _stream_ptr(stream))
    _check(h, rc)
    return idx, dist, acc


def latch_detect(h, img, threshold, max_kps, kps=None, n_kps=None, image_id=None, image_index=0,
                 stream=None):
    """FAST-9 keypoints with orientation, appended to kps after the n_kps[0]
    already there; returns (kps float32 [max_kps, 4], n_kps int64 [1] on the
    device: the new total, which may exceed max_kps).  A new n_kps starts at 0."""
    import torch
    if img.dim() != 2:
        raise ValueError("img must be 2-D")
    dev = img.device
    if kps is None:
        kps = torch.empty((max_kps, 4), dtype=torch.float32, device=dev)
    if n_kps is None:
        n_kps = torch.zeros((1,), dtype=torch.int64, device=dev)
    H, W = img.shape
    idp = _dev(image_id, torch.int32, "image_id") if image_id is not None else None
    args = (h, _dev(img, torch.uint8, "img"), H, W, img.stride(0), int(threshold),
            _dev(kps, torch.float32, "kps"), int(max_kps), _dev(n_kps, torch.int64, "n_kps"), idp,
            int(image_index), _stream_ptr(stream))
    _with_workspace(h, lambda: load_library().latch_detect(*args),
                    lambda: latch_detect_workspace_size(h, H, W))
    return kps, n_kps


IMAGE_ENTRY_BYTES = 24


def image_table(images):
    """Pack device images (uint8 CUDA tensors [H, W], row stride = pitch) into a
    latch_image table: a uint8 CUDA tensor of n * 24 bytes."""
    import torch
    rows = np.zeros((len(images), 3), np.int64)
    for i, img in enumerate(images):
        if img.dim() != 2 or img.dtype != torch.uint8 or not img.is_cuda or img.stride(1) != 1:
            raise TypeError("images must be 2-D uint8 CUDA tensors with unit column stride")
        H, W = img.shape
        rows[i, 0] = img.data_ptr()
        rows[i, 1] = H | (W << 32)
        rows[i, 2] = img.stride(0)
    return torch.from_numpy(rows.view(np.uint8).reshape(-1)).to(images[0].device)


def latch_extract_batch(h, table, n_images, image_id, kps, desc=None, n_kps=None, stream=None):
    """Batched extraction.  table: from image_table(); image_id: int32 [n] CUDA;
    kps: float32 [n, 4] CUDA; n_kps: optional int64 [1] CUDA tensor (count to process)."""
    import torch
    n = kps.shape[0]
    if image_id.shape[0] != n:
        raise ValueError("image_id must have one entry per keypoint")
    if desc is None:
        desc = torch.empty((n, 16), dtype=torch.int32, device=kps.device)
    nptr = _dev(n_kps, torch.int64, "n_kps") if n_kps is not None else None
    args = (h, _dev(table, torch.uint8, "table"), int(n_images),
            _dev(image_id, torch.int32, "image_id"), _dev(kps, torch.float32, "kps"), n, nptr,
            _dev(desc, torch.int32, "desc"), _stream_ptr(stream))
    _with_workspace(h, lambda: load_library().latch_extract_batch(*args),
                    lambda: latch_extract_batch_workspace_size(h, n_images, n))
    return desc


def hamming_knn(h, query, train, k=2, ratio=0.8, path="auto", idx=None, dist=None, accept=None,
                want_accept=True, stream=None):
    """Brute-force k-NN.  query [nq, 16], train [nt, 16] int32 (uint32 bit patterns).

    Returns (idx int32 [nq, k], dist int32 [nq, k], accept uint8 [nq] or None)."""
    import torch
    nq, nt = query.shape[0], train.shape[0]
    dev = query.device
    if idx is None:
        idx = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if dist is None:
        dist = torch.empty((nq, k), dtype=torch.int32, device=dev)
    if accept is None and want_accept:
        accept = torch.empty((nq,), dtype=torch.uint8, device=dev)
    acc_ptr = _dev(accept, torch.uint8, "accept") if accept is not None else None
    tptr = _dev(train, torch.int32, "train") if nt > 0 else None
    args = (h, _dev(query, torch.int32, "query"), nq, tptr, nt, int(k), float(ratio),
            _dev(idx, torch.int32, "idx"), _dev(dist, torch.int32, "dist"), acc_ptr, PATHS[path],
            _stream_ptr(stream))
    _with_workspace(h, lambda: load_library().hamming_knn(*args),
                    lambda: hamming_knn_workspace_size(h, nq, nt, path))
    return idx, dist, accept


def hamming_knn_noalloc(h, query, train, idx, dist, accept=None, k=2, ratio=0.8, path="auto",
                        stream=None):
    """hamming_knn with its split partials in the library's static device
    scratch: the caller passes every output (idx, dist int32 [nq, k], accept
    uint8 [nq] or None) and nothing is allocated."""
    import torch
    nq, nt = query.shape[0], train.shape[0]
    acc_ptr = _dev(accept, torch.uint8, "accept") if accept is not None else None
    tptr = _dev(train, torch.int32, "train") if nt > 0 else None
    _check(h, load_library().hamming_knn_noalloc(
        h, _dev(query, torch.int32, "query"), nq, tptr, nt, int(k), float(ratio),
        _dev(idx, torch.int32, "idx"), _dev(dist, torch.int32, "dist"), acc_ptr, PATHS[path],
        _stream_ptr(stream)))
    return idx, dist, accept


NOALLOC_SCRATCH_BYTES = 16 << 20     # LATCH_NOALLOC_SCRATCH_BYTES


def pair_table(pairs, device="cuda"):
    """latch_pair table from rows (query_first, nq, train_first, nt, out_first):
    an int64 CUDA tensor [n, 5]."""
    import torch
    arr = np.asarray(pairs, np.int64).reshape(-1, 5)
    return torch.from_numpy(np.ascontiguousarray(arr)).to(device)


def hamming_knn_batch(h, query, train, pairs, out_rows, k=2, ratio=0.8, path="auto", idx=None,
                      dist=None, accept=None, want_accept=True, stream=None):
    """Batched k-NN over a pair table (see pair_table).  Returns (idx, dist, accept)
    with out_rows rows; rows no pair writes are left as allocated."""
    import torch
    dev = query.device
    if idx is None:
        idx = torch.full((out_rows, k), -2, dtype=torch.int32, device=dev)
    if dist is None:
        dist = torch.full((out_rows, k), -2, dtype=torch.int32, device=dev)
    if accept is None and want_accept:
        accept = torch.full((out_rows,), 255, dtype=torch.uint8, device=dev)
    acc_ptr = _dev(accept, torch.uint8, "accept") if accept is not None else None
    qptr = _dev(query, torch.int32, "query") if query.shape[0] else None
    tptr = _dev(train, torch.int32, "train") if train.shape[0] else None
    args = (h, qptr, query.shape[0], tptr, train.shape[0], _dev(pairs, torch.int64, "pairs"),
            pairs.shape[0], int(k), float(ratio), _dev(idx, torch.int32, "idx"),
            _dev(dist, torch.int32, "dist"), acc_ptr, int(out_rows), PATHS[path], _stream_ptr(stream))
    _with_workspace(h, lambda: load_library().hamming_knn_batch(*args),
                    lambda: hamming_knn_batch_workspace_size(h, pairs.shape[0], out_rows))
    return idx, dist, accept


class Tuning(ctypes.Structure):
    """latch_tuning: path per (bucket(nq), bucket(nt)), batch path, split targets."""
    _fields_ = [("path", (ctypes.c_int8 * 8) * 8), ("batch_path", ctypes.c_int8),
                ("fp4_query_blocks", ctypes.c_int8), ("reserved", ctypes.c_int8 * 2),
                ("mfma_groups_per_cu", ctypes.c_int32),
                ("popcount_groups_per_cu", ctypes.c_int32), ("batch_groups_per_cu", ctypes.c_int32)]

    SCALARS = ("batch_path", "fp4_query_blocks", "mfma_groups_per_cu", "popcount_groups_per_cu",
               "batch_groups_per_cu")
    DEFAULTS = {"fp4_query_blocks": 3, "batch_groups_per_cu": 2}

    def to_dict(self):
        d = {"path": [[int(self.path[i][j]) for j in range(8)] for i in range(8)]}
        d.update({k: int(getattr(self, k)) for k in self.SCALARS})
        return d

    @classmethod
    def from_dict(cls, d):
        """A latch_tuning from a dict; fields missing from older tables take
        the library defaults."""
        t = cls()
        for i in range(8):
            for j in range(8):
                t.path[i][j] = d["path"][i][j]
        for k in cls.SCALARS:
            setattr(t, k, d.get(k, cls.DEFAULTS.get(k, 0)))
        return t


def size_bucket(n):
    """Bucket of a size for the tuning table: min(7, floor(log2(max(n, 1)) / 2))."""
    b = 0
    while b < 7 and (int(n) >> (2 * (b + 1))) > 0:
        b += 1
    return b


def latch_get_tuning(h):
    t = Tuning()
    _check(h, load_library().latch_get_tuning(h, ctypes.byref(t)))
    return t


def latch_set_tuning(h, t):
    _check(h, load_library().latch_set_tuning(h, ctypes.byref(t)))


class _PlanDesc(ctypes.Structure):
    _fields_ = [("images", ctypes.c_void_p), ("n_images", ctypes.c_int32),
                ("image_id", ctypes.c_void_p), ("kps", ctypes.c_void_p),
                ("n_kps", ctypes.c_void_p), ("max_kps", ctypes.c_int64),
                ("desc", ctypes.c_void_p), ("pairs", ctypes.c_void_p),
                ("n_pairs", ctypes.c_int32), ("k", ctypes.c_int32), ("ratio", ctypes.c_float),
                ("path", ctypes.c_int32), ("idx", ctypes.c_void_p), ("dist", ctypes.c_void_p),
                ("accept", ctypes.c_void_p), ("out_rows", ctypes.c_int64)]


class Plan:
    """A captured batched extract + match graph (latch_plan_*).  Holds references
    to the device tensors whose pointers the graph uses."""

    def __init__(self, h, table, n_images, image_id, kps, desc, pairs, idx, dist, accept=None,
                 n_kps=None, k=2, ratio=0.8, path="auto"):
        import torch
        self._keep = (table, image_id, kps, desc, pairs, idx, dist, accept, n_kps)
        d = _PlanDesc()
        d.images = _dev(table, torch.uint8, "table").value
        d.n_images = n_images
        d.image_id = _dev(image_id, torch.int32, "image_id").value
        d.kps = _dev(kps, torch.float32, "kps").value
        d.n_kps = _dev(n_kps, torch.int64, "n_kps").value if n_kps is not None else None
        d.max_kps = kps.shape[0]
        d.desc = _dev(desc, torch.int32, "desc").value
        d.pairs = _dev(pairs, torch.int64, "pairs").value
        d.n_pairs = pairs.shape[0]
        d.k, d.ratio, d.path = k, float(ratio), PATHS[path]
        d.idx = _dev(idx, torch.int32, "idx").value
        d.dist = _dev(dist, torch.int32, "dist").value
        d.accept = _dev(accept, torch.uint8, "accept").value if accept is not None else None
        d.out_rows = idx.shape[0]
        self.h = h
        self.p = ctypes.c_void_p()
        _check(h, load_library().latch_plan_create(h, ctypes.byref(d), ctypes.byref(self.p)))

    def run(self, stream=None):
        _check(self.h, load_library().latch_plan_run(self.p, _stream_ptr(stream)))

    def close(self):
        if self.p:
            load_library().latch_plan_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def latch_check_errors(h, stream=None, clear=True):
    v = ctypes.c_uint32()
    rc = load_library().latch_check_errors(h, _stream_ptr(stream), ctypes.byref(v), int(clear))
    _check(h, rc)
    return v.value


def latch_timing_enable(h, enable=True):
    _check(h, load_library().latch_timing_enable(h, int(bool(enable))))


def latch_timing_read(h, kernel):
    """(launches, total_ms) recorded for one kernel name since timing was enabled."""
    n = ctypes.c_int()
    ms = ctypes.c_double()
    _check(h, load_library().latch_timing_read(h, kernel.encode(), ctypes.byref(n),
                                               ctypes.byref(ms)))
    return n.value, ms.value


class Latch:
    """Owning wrapper of a handle (the same calls, with the handle bound)."""

    def __init__(self, triplets, window=None, patch=None, weights=None):
        """The default geometry (48 x 48 window, 7 x 7 patches, unit weights),
        or another one (latch_create_geometry) when any of window, patch or
        weights is given."""
        if window is None and patch is None and weights is None:
            self.h = latch_create(triplets)
        else:
            self.h = latch_create_geometry(triplets, window or 48, patch or 7, weights)

    def extract(self, img, kps, desc=None, stream=None):
        return latch_extract(self.h, img, kps, desc, stream)

    def extract_dense(self, img, x0, y0, gw, gh, desc=None, stream=None):
        return latch_extract_dense(self.h, img, x0, y0, gw, gh, desc, stream)

    def knn_window(self, query, train, gw, gh, radius, k=2, ratio=0.8, stream=None):
        return hamming_knn_window(self.h, query, train, gw, gh, radius, k, ratio, stream)

    def detect(self, img, threshold, max_kps, **kw):
        return latch_detect(self.h, img, threshold, max_kps, **kw)

    def extract_batch(self, table, n_images, image_id, kps, desc=None, n_kps=None, stream=None):
        return latch_extract_batch(self.h, table, n_images, image_id, kps, desc, n_kps, stream)

    def reserve(self, nbytes=0):
        return latch_reserve(self.h, nbytes)

    def knn_workspace_size(self, nq, nt, path="auto"):
        return hamming_knn_workspace_size(self.h, nq, nt, path)

    def knn_batch_workspace_size(self, n_pairs, out_rows):
        return hamming_knn_batch_workspace_size(self.h, n_pairs, out_rows)

    def detect_workspace_size(self, height, width):
        return latch_detect_workspace_size(self.h, height, width)

    def extract_batch_workspace_size(self, n_images, max_kps):
        return latch_extract_batch_workspace_size(self.h, n_images, max_kps)

    def knn(self, query, train, k=2, ratio=0.8, path="auto", **kw):
        return hamming_knn(self.h, query, train, k, ratio, path, **kw)

    def knn_batch(self, query, train, pairs, out_rows, k=2, ratio=0.8, path="auto", **kw):
        return hamming_knn_batch(self.h, query, train, pairs, out_rows, k, ratio, path, **kw)

    def get_tuning(self):
        return latch_get_tuning(self.h)

    def set_tuning(self, t):
        latch_set_tuning(self.h, t)

    def plan(self, *args, **kw):
        return Plan(self.h, *args, **kw)

    def check_errors(self, stream=None, clear=True):
        return latch_check_errors(self.h, stream, clear)

    def timing(self, enable=True):
        latch_timing_enable(self.h, enable)

    def timing_read(self, kernel):
        return latch_timing_read(self.h, kernel)

    def close(self):
        if self.h is not None:
            latch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
