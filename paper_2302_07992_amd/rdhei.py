"""Python binding of librdhei (argument marshalling only).

Every stage runs in the HIP library; this module converts torch tensors to
device pointers and forwards to the C ABI declared in ``include/rdhei.h``.
Importing it without a built ``librdhei.so`` raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librdhei.so")

OK, EINVAL, ECAPACITY, ENOFIT, ENOMEM, EDEVICE, ECORRUPT = 0, -1, -2, -3, -4, -5, -6
EMR, LMR, DEMR = 0, 1, 2
OP_ENCRYPT, OP_EMBED, OP_EXTRACT, OP_RECOVER = 0, 1, 2, 3
PLAN_GRAPH, PLAN_EAGER, PLAN_PER_IMAGE = 0, 1, 2
TUNE_FORCE = 1
OPT_PER_PIXEL, OPT_MAX_GRID, OPT_RESERVE_WS, OPT_HIDE_MODE, OPT_LMR_MIN_LEVEL, OPT_KEYSTREAM = 1, 2, 3, 4, 5, 6
OPT_QUAD_SEG = 7
OPT_WG_PER_IMAGE = 8
KEYSTREAM_PHILOX, KEYSTREAM_CHACHA20 = 0, 1
META_BYTES = 64

EXPORTS = [
    "rdhei_ctx_create", "rdhei_ctx_destroy", "rdhei_ctx_set_option",
    "rdhei_encrypt", "rdhei_embed", "rdhei_extract", "rdhei_recover",
    "rdhei_workspace_size", "rdhei_run_batch", "rdhei_run_batch_static",
    "rdhei_roles_workspace_size", "rdhei_run_roles", "rdhei_plan_create", "rdhei_plan_run", "rdhei_plan_destroy", "rdhei_plan_set_grid",
    "rdhei_plan_stage_count", "rdhei_plan_stage_name", "rdhei_plan_run_stage",
    "rdhei_plan_autotune", "rdhei_plan_stage_grid", "rdhei_plan_tuned", "rdhei_ctx_set_tune_file",
    "rdhei_lmr_batch", "rdhei_lmr_compress", "rdhei_lmr_decompress", "rdhei_metrics", "rdhei_tile_b",
    "rdhei_strerror", "rdhei_last_error", "rdhei_version",
]


class RdheiError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(what)


class MetaStruct(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32), ("method", ctypes.c_int32),
                ("b", ctypes.c_int32), ("min_level", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("redundant", ctypes.c_int64), ("capacity_bits", ctypes.c_int64), ("map_bits", ctypes.c_int64),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32), ("nonce", ctypes.c_uint64)]


assert ctypes.sizeof(MetaStruct) == META_BYTES


class MetricJobStruct(ctypes.Structure):
    """rdhei_metric_job: one image pair of rdhei_metrics (device pointers)."""
    _fields_ = [("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("height", ctypes.c_int32),
                ("width", ctypes.c_int32)]


METRIC_COUNT, METRIC_SSIM = 8, 1
METRIC_NAMES = ("entropy_a", "chi2_a", "entropy_b", "chi2_b", "npcr", "uaci", "psnr", "ssim")


class JobStruct(ctypes.Structure):
    _fields_ = [("inp", ctypes.c_void_p), ("out", ctypes.c_void_p), ("msg", ctypes.c_void_p),
                ("meta", ctypes.c_void_p), ("key", ctypes.c_uint64), ("nonce", ctypes.c_uint64),
                ("nbits", ctypes.c_int64),
                ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("method", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("btab", ctypes.c_void_p)]


# numpy view of rdhei_job, for building large job tables without Python loops
JOB_DTYPE = np.dtype([("inp", "<u8"), ("out", "<u8"), ("msg", "<u8"), ("meta", "<u8"), ("key", "<u8"),
                      ("nonce", "<u8"), ("nbits", "<i8"), ("height", "<i4"), ("width", "<i4"), ("method", "<i4"),
                      ("reserved", "<i4"), ("btab", "<u8")])
assert JOB_DTYPE.itemsize == ctypes.sizeof(JobStruct)


def _jobs_arg(jobs):
    """(pointer, count) of a job table given as a ctypes array or a JOB_DTYPE array."""
    if isinstance(jobs, np.ndarray):
        if jobs.dtype != JOB_DTYPE or not jobs.flags.c_contiguous:
            raise TypeError("job table must be a contiguous JOB_DTYPE array")
        return jobs.ctypes.data_as(ctypes.POINTER(JobStruct)), len(jobs)
    return jobs, len(jobs)


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librdhei.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"librdhei.so not found at {path}: build it with "
                           "`python -m paper_2302_07992_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    lib.rdhei_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.rdhei_ctx_destroy.argtypes = [vp]
    lib.rdhei_ctx_destroy.restype = None
    lib.rdhei_ctx_set_option.argtypes = [vp, i32, i64]
    lib.rdhei_encrypt.argtypes = [vp, vp, vp, i32, i32, u64, u64, i32, vp, vp]
    lib.rdhei_embed.argtypes = [vp, vp, i32, i32, i32, vp, vp, i64, u64, vp]
    lib.rdhei_extract.argtypes = [vp, vp, i32, i32, i32, vp, vp, i64, u64, vp]
    lib.rdhei_recover.argtypes = [vp, vp, i32, i32, i32, vp, vp, u64, vp]
    lib.rdhei_workspace_size.argtypes = [vp, i32, ctypes.POINTER(JobStruct), i32, ctypes.POINTER(ctypes.c_int64)]
    lib.rdhei_run_batch.argtypes = [vp, i32, ctypes.POINTER(JobStruct), i32, vp, ctypes.c_int64, vp]
    lib.rdhei_run_batch_static.argtypes = [vp, i32, ctypes.POINTER(JobStruct), i32, vp]
    lib.rdhei_roles_workspace_size.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(i32),
                                               ctypes.POINTER(ctypes.c_int64)]
    lib.rdhei_run_roles.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(i32), vp,
                                    ctypes.c_int64, vp]
    lib.rdhei_plan_create.argtypes = [vp, i32, ctypes.POINTER(JobStruct), i32, i32, ctypes.POINTER(vp)]
    lib.rdhei_plan_run.argtypes = [vp, vp]
    lib.rdhei_plan_destroy.argtypes = [vp]
    lib.rdhei_plan_destroy.restype = None
    lib.rdhei_plan_set_grid.argtypes = [vp, i32]
    lib.rdhei_plan_stage_count.argtypes = [vp]
    lib.rdhei_plan_stage_name.argtypes = [vp, i32]
    lib.rdhei_plan_stage_name.restype = ctypes.c_char_p
    lib.rdhei_plan_run_stage.argtypes = [vp, i32, vp]
    lib.rdhei_plan_autotune.argtypes = [vp, i32, i32, vp]
    lib.rdhei_plan_stage_grid.argtypes = [vp, i32]
    lib.rdhei_plan_tuned.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.rdhei_ctx_set_tune_file.argtypes = [vp, ctypes.c_char_p]
    lib.rdhei_lmr_batch.argtypes = [vp, i32, ctypes.POINTER(JobStruct), i32, i32, ctypes.POINTER(ctypes.c_double), vp]
    lib.rdhei_lmr_compress.argtypes = [vp, vp, i32, i32, vp, i64, ctypes.POINTER(i64)]
    lib.rdhei_lmr_decompress.argtypes = [vp, i64, i32, i32, vp, vp]
    lib.rdhei_metrics.argtypes = [vp, ctypes.POINTER(MetricJobStruct), i32, i32, vp, vp]
    lib.rdhei_tile_b.argtypes = [vp, ctypes.POINTER(MetricJobStruct), i32, vp, vp, vp]
    lib.rdhei_strerror.argtypes = [ctypes.c_int]
    lib.rdhei_strerror.restype = ctypes.c_char_p
    lib.rdhei_last_error.argtypes = []
    lib.rdhei_last_error.restype = ctypes.c_char_p
    lib.rdhei_version.argtypes = []
    lib.rdhei_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != OK:
        lib = load_library()
        raise RdheiError(rc, f"{what}: {lib.rdhei_strerror(rc).decode()} {lib.rdhei_last_error().decode()}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def msg_bytes(nbits: int) -> int:
    """Bytes a message buffer needs: ceil(nbits / 128) * 16 (at least 16)."""
    return max(16, (nbits + 127) // 128 * 16)


def new_meta(n: Optional[int] = None, device="cuda") -> torch.Tensor:
    shape = (META_BYTES,) if n is None else (n, META_BYTES)
    return torch.zeros(shape, dtype=torch.uint8, device=device)


@dataclass
class Meta:
    height: int
    width: int
    method: int
    b: int
    min_level: int
    max_level: int
    redundant: int
    capacity_bits: int
    map_bits: int
    status: int
    nonce: int = 0


def read_meta(t: torch.Tensor):
    """Decode one (64,) or many (n, 64) meta records (copies to host)."""
    a = t.detach().to("cpu").contiguous().numpy()
    rows = a.reshape(-1, META_BYTES)
    out = []
    for r in rows:
        m = MetaStruct.from_buffer_copy(r.tobytes())
        out.append(Meta(m.height, m.width, m.method, m.b, m.min_level, m.max_level, m.redundant,
                        m.capacity_bits, m.map_bits, m.status, m.nonce))
    return out[0] if a.ndim == 1 else out


def read_meta_array(t: torch.Tensor) -> np.ndarray:
    """Vectorised decode of (n, 64) metas: structured numpy array."""
    dt = np.dtype([("height", "<i4"), ("width", "<i4"), ("method", "<i4"), ("b", "<i4"), ("min_level", "<i4"),
                   ("max_level", "<i4"), ("redundant", "<i8"), ("capacity_bits", "<i8"), ("map_bits", "<i8"),
                   ("status", "<i4"), ("reserved", "<i4"), ("nonce", "<u8")])
    return t.detach().to("cpu").contiguous().numpy().reshape(-1).view(dt)


class Context:
    """A librdhei context on one GPU (owns the single-image workspace)."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        h = ctypes.c_void_p()
        _check(self.lib.rdhei_ctx_create(ctypes.byref(h), device), "rdhei_ctx_create")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.lib.rdhei_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option: int, value: int) -> None:
        _check(self.lib.rdhei_ctx_set_option(self.h, option, value), "rdhei_ctx_set_option")

    def set_tune_file(self, path) -> None:
        """Persist the autotuner's choices in a JSON file (loaded now if it
        exists, rewritten after every autotune); None: memory only."""
        _check(self.lib.rdhei_ctx_set_tune_file(self.h, None if path is None else str(path).encode()),
               "rdhei_ctx_set_tune_file")

    def encrypt(self, img: torch.Tensor, enc: torch.Tensor, k1: int, meta: torch.Tensor, method: int = EMR,
                stream=None, nonce: int = 0) -> None:
        """Content owner: encrypt `img` into `enc` with key k1 and the image's
        keystream nonce (recorded in `meta` for the other roles)."""
        M, N = img.shape
        _check(self.lib.rdhei_encrypt(self.h, _ptr(img), _ptr(enc), M, N, k1, nonce, method, _ptr(meta),
                                      _stream(stream)), "rdhei_encrypt")

    def embed(self, marked: torch.Tensor, meta: torch.Tensor, msg: torch.Tensor, nbits: int, k2: int,
              method: int = EMR, stream=None) -> None:
        M, N = marked.shape
        _check(self.lib.rdhei_embed(self.h, _ptr(marked), M, N, method, _ptr(meta), _ptr(msg), nbits, k2,
                                    _stream(stream)), "rdhei_embed")

    def extract(self, marked: torch.Tensor, meta: torch.Tensor, msg: torch.Tensor, nbits: int, k2: int,
                method: int = EMR, stream=None) -> None:
        M, N = marked.shape
        _check(self.lib.rdhei_extract(self.h, _ptr(marked), M, N, method, _ptr(meta), _ptr(msg), nbits, k2,
                                      _stream(stream)), "rdhei_extract")

    def workspace_size(self, op: int, jobs) -> int:
        """Device workspace bytes that run_batch needs for this op and job array."""
        out = ctypes.c_int64(0)
        p, n = _jobs_arg(jobs)
        _check(self.lib.rdhei_workspace_size(self.h, op, p, n, ctypes.byref(out)), "rdhei_workspace_size")
        return int(out.value)

    def run_batch(self, op: int, jobs, workspace_ptr: int = 0, workspace_bytes: int = 0, stream=None) -> None:
        """One EMR op over a job array (see make_jobs), launched directly on
        `stream`; workspace_ptr 0 uses the context's own workspace."""
        p, n = _jobs_arg(jobs)
        _check(self.lib.rdhei_run_batch(self.h, op, p, n, ctypes.c_void_p(workspace_ptr or None),
                                        workspace_bytes, _stream(stream)), "rdhei_run_batch")

    @staticmethod
    def _roles_args(roles):
        """(n, ops, tables, counts) C arrays of [(op, job table), ...]; the
        tables (ctypes arrays or JOB_DTYPE arrays) must stay alive meanwhile."""
        n = len(roles)
        ops = (ctypes.c_int32 * n)(*[int(op) for op, _ in roles])
        tabs = (ctypes.c_void_p * n)()
        cnt = (ctypes.c_int32 * n)()
        for i, (_, t) in enumerate(roles):
            if isinstance(t, np.ndarray):
                if t.dtype != JOB_DTYPE or not t.flags.c_contiguous:
                    raise TypeError("job table must be a contiguous JOB_DTYPE array")
                tabs[i] = t.ctypes.data
            else:
                tabs[i] = ctypes.addressof(t)
            cnt[i] = len(t)
        return n, ops, tabs, cnt

    def roles_workspace_size(self, roles) -> int:
        """Workspace bytes of run_roles over [(op, job table), ...]."""
        n, ops, tabs, cnt = self._roles_args(roles)
        out = ctypes.c_int64(0)
        _check(self.lib.rdhei_roles_workspace_size(self.h, n, ops, tabs, cnt, ctypes.byref(out)),
               "rdhei_roles_workspace_size")
        return int(out.value)

    def run_roles(self, roles, workspace_ptr: int = 0, workspace_bytes: int = 0, stream=None) -> None:
        """Several EMR ops of one batch, [(op, job table), ...], in order on
        `stream` with one table upload (rdhei_run_roles)."""
        n, ops, tabs, cnt = self._roles_args(roles)
        _check(self.lib.rdhei_run_roles(self.h, n, ops, tabs, cnt, ctypes.c_void_p(workspace_ptr or None),
                                        workspace_bytes, _stream(stream)), "rdhei_run_roles")

    def run_batch_static(self, op: int, jobs, stream=None) -> None:
        """One EMR op over a job array with the library's static device
        scratch (rdhei_run_batch_static: no allocation)."""
        p, n = _jobs_arg(jobs)
        _check(self.lib.rdhei_run_batch_static(self.h, op, p, n, _stream(stream)), "rdhei_run_batch_static")

    def metrics(self, pairs, ssim: bool = True, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Sec. IV image metrics of each (a, b) pair (b may be None), or of a
        job array from make_metric_jobs: a device tensor of shape (n, 8),
        columns as METRIC_NAMES.  Asynchronous."""
        jobs = pairs if isinstance(pairs, ctypes.Array) else make_metric_jobs(pairs)
        n = len(jobs)
        if out is None:
            dev = pairs[0][0].device if not isinstance(pairs, ctypes.Array) else torch.device("cuda")
            out = torch.empty((n, METRIC_COUNT), dtype=torch.float64, device=dev)
        _check(self.lib.rdhei_metrics(self.h, jobs, n, METRIC_SSIM if ssim else 0, ctypes.c_void_p(out.data_ptr()),
                                      _stream(stream)), "rdhei_metrics")
        return out

    def tile_b(self, images, stream=None):
        """Per-tile b of each image (contiguous 2-D uint8 device tensors, sides
        multiples of 64; rdhei_tile_b): (tile_b, capacity) device tensors, one
        byte per 64x64 tile of every image in order (row-major) and one int64
        capacity in bits per image.  Asynchronous."""
        jobs = make_metric_jobs([(x, None) for x in images])
        n = len(jobs)
        ntiles = sum((int(x.shape[0]) // 64) * (int(x.shape[1]) // 64) for x in images)
        dev = images[0].device
        tb = torch.empty(max(ntiles, 1), dtype=torch.uint8, device=dev)
        cap = torch.empty(n, dtype=torch.int64, device=dev)
        _check(self.lib.rdhei_tile_b(self.h, jobs, n, ctypes.c_void_p(tb.data_ptr()), ctypes.c_void_p(cap.data_ptr()),
                                     _stream(stream)), "rdhei_tile_b")
        return tb[:ntiles], cap

    def lmr_batch(self, op: int, jobs, threads: int = 0, stream=None) -> dict:
        """One LMR role over a job array (method LMR); returns the seconds spent
        in device stages, in the host coder and in total."""
        p, n = _jobs_arg(jobs)
        t = (ctypes.c_double * 3)()
        _check(self.lib.rdhei_lmr_batch(self.h, op, p, n, threads, t, _stream(stream)), "rdhei_lmr_batch")
        return {"device_s": t[0], "coder_s": t[1], "total_s": t[2]}

    def recover(self, marked: torch.Tensor, meta: torch.Tensor, out: torch.Tensor, k1: int, method: int = EMR,
                stream=None) -> None:
        M, N = marked.shape
        _check(self.lib.rdhei_recover(self.h, _ptr(marked), M, N, method, _ptr(meta), _ptr(out), k1,
                                      _stream(stream)), "rdhei_recover")


def make_metric_jobs(pairs) -> ctypes.Array:
    """rdhei_metric_job array from (a, b) pairs of contiguous 2-D uint8
    device tensors (b may be None)."""
    n = len(pairs)
    arr = (MetricJobStruct * n)()
    for i, (a, b) in enumerate(pairs):
        if a.dtype != torch.uint8 or a.dim() != 2 or not a.is_contiguous():
            raise RdheiError(EINVAL, "metrics: images must be contiguous 2-D uint8 tensors")
        if b is not None and (b.shape != a.shape or b.dtype != torch.uint8 or not b.is_contiguous()):
            raise RdheiError(EINVAL, "metrics: b must match a")
        arr[i].a = a.data_ptr()
        arr[i].b = b.data_ptr() if b is not None else None
        arr[i].height, arr[i].width = int(a.shape[0]), int(a.shape[1])
    return arr


def make_jobs(ins: Sequence, outs: Sequence, msgs: Sequence, metas: Sequence, keys: Sequence[int],
              nbits: Sequence[int], shapes: Sequence, method: int = EMR, nonces: Optional[Sequence[int]] = None,
              btabs: Optional[Sequence] = None):
    """Job array from per-image pointers (ints) or tensors (None allowed);
    nonces: per-image keystream nonces of an ENCRYPT batch (default 0);
    btabs: DEMR tile b tables (device, (height/64) * (width/64) bytes each)."""
    n = len(keys)
    arr = (JobStruct * n)()

    def p(x):
        if x is None:
            return None
        return x if isinstance(x, int) else x.data_ptr()

    for i in range(n):
        arr[i].inp = p(ins[i]) if ins is not None else None
        arr[i].out = p(outs[i]) if outs is not None else None
        arr[i].msg = p(msgs[i]) if msgs is not None else None
        arr[i].meta = p(metas[i])
        arr[i].key = int(keys[i]) & ((1 << 64) - 1)
        arr[i].nonce = (int(nonces[i]) & ((1 << 64) - 1)) if nonces is not None else 0
        arr[i].nbits = int(nbits[i]) if nbits is not None else 0
        arr[i].height, arr[i].width = int(shapes[i][0]), int(shapes[i][1])
        arr[i].method = method
        arr[i].reserved = 0
        arr[i].btab = p(btabs[i]) if btabs is not None else None
    return arr


class Plan:
    """A reusable batched launch of one op (graph-captured by default)."""

    def __init__(self, ctx: Context, op: int, jobs, flags: int = PLAN_GRAPH):
        self.lib = ctx.lib
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(self.lib.rdhei_plan_create(ctx.h, op, jobs, len(jobs), flags, ctypes.byref(h)), "rdhei_plan_create")
        self.h = h
        self.jobs = jobs

    def set_grid(self, max_workgroups: int) -> None:
        _check(self.lib.rdhei_plan_set_grid(self.h, max_workgroups), "rdhei_plan_set_grid")

    def run(self, stream=None) -> None:
        _check(self.lib.rdhei_plan_run(self.h, _stream(stream)), "rdhei_plan_run")

    def stages(self):
        n = self.lib.rdhei_plan_stage_count(self.h)
        return [self.lib.rdhei_plan_stage_name(self.h, k).decode() for k in range(n)]

    def run_stage(self, k: int, stream=None) -> None:
        _check(self.lib.rdhei_plan_run_stage(self.h, k, _stream(stream)), "rdhei_plan_run_stage")

    def autotune(self, reps: int = 3, force: bool = False, stream=None) -> list:
        """Pick each stage's workgroup count by timing (see rdhei_plan_autotune);
        returns the chosen counts (0 = the launcher's default)."""
        _check(self.lib.rdhei_plan_autotune(self.h, reps, TUNE_FORCE if force else 0, _stream(stream)),
               "rdhei_plan_autotune")
        return self.stage_grids()

    def tuned(self) -> dict:
        """The plan's layout variant: hiding mode, quads per work unit, workgroup-per-image mode."""
        hm, qs, wi = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.rdhei_plan_tuned(self.h, ctypes.byref(hm), ctypes.byref(qs), ctypes.byref(wi)),
               "rdhei_plan_tuned")
        return {"hide_mode": hm.value, "qseg": qs.value, "wg_image": wi.value}

    def stage_grids(self) -> list:
        return [int(self.lib.rdhei_plan_stage_grid(self.h, k)) for k in range(self.lib.rdhei_plan_stage_count(self.h))]

    def close(self):
        if getattr(self, "h", None):
            self.lib.rdhei_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lmr_compress(eta_bits: np.ndarray, l_bits: np.ndarray, M: int, N: int, capacity_bytes: int):
    """Host map coder: returns (stream bytes, stream bits) or raises RdheiError(ENOFIT)."""
    lib = load_library()
    eta = np.ascontiguousarray(eta_bits, dtype=np.uint8)
    lb = np.ascontiguousarray(l_bits, dtype=np.uint8)
    out = np.zeros(max(capacity_bytes, 8) + 16, dtype=np.uint8)
    bits = ctypes.c_int64()
    rc = lib.rdhei_lmr_compress(eta.ctypes.data, lb.ctypes.data, M, N, out.ctypes.data, capacity_bytes,
                                ctypes.byref(bits))
    _check(rc, "rdhei_lmr_compress")
    return out[: bits.value // 8].copy(), bits.value


def lmr_decompress(stream: np.ndarray, M: int, N: int):
    lib = load_library()
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    nb = (M * N + 7) // 8
    eta = np.zeros(nb + 16, dtype=np.uint8)
    lb = np.zeros(nb + 16, dtype=np.uint8)
    _check(lib.rdhei_lmr_decompress(s.ctypes.data, s.size, M, N, eta.ctypes.data, lb.ctypes.data),
           "rdhei_lmr_decompress")
    return eta[:nb], lb[:nb]
