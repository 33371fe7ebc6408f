"""Python binding of libccpt (include/ccpt.h): argument marshalling only.

PyTorch supplies device memory and streams; every step of the tracking
path runs in the library's HIP kernels.  Loading fails loudly when the
library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_size_t, c_void_p

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccpt.so")

# return codes
OK = 0
E_INVALID = -1
E_UNSUPPORTED = -2
E_NOREF = -3
E_HIP = -4
E_NONPOSITIVE_REF = -5
E_NOMEM = -6

# status bits
ST_NONFINITE = 1
ST_FLAT = 2
ST_NEAR_TIE = 4
ST_NEWTON_FALLBACK = 8
ST_WINDOW_EXIT = 16

MODES = {"ccu": 0, "ccsn": 1}
PRECISIONS = {"fp32": 0, "bf16x2": 1, "fp16x2": 2, "fp64": 3}
U16, F32, F64 = 0, 1, 2
FLAG_GRAPH = 1
FLAG_PROFILE = 2
FLAG_STREAMS = 4
STAGES = ["init", "rows_fwd", "cols", "rows_inv", "updft", "newton", "grad", "xcorr"]

RESULT_DTYPE = np.dtype([
    ("d", "<f8", (2,)),
    ("peak", "<f8"),
    ("hess", "<f8", (3,)),
    ("d_grid", "<f4", (2,)),
    ("p", "<i4", (2,)),
    ("status", "<u4"),
    ("reserved", "<u4"),
])
RESULT_BYTES = RESULT_DTYPE.itemsize  # 72


class Options(ctypes.Structure):
    _fields_ = [("mode", c_int), ("eps", c_double), ("upsample", c_int), ("window", c_double),
                ("precision", c_int), ("newton_iters", c_int), ("flags", c_int)]


class Image(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("ny", c_int), ("nx", c_int), ("pitch", c_int), ("dtype", c_int)]


class Plan(ctypes.Structure):
    _fields_ = [("chunk", c_int), ("split_blocks", c_int), ("fused_min", c_int)]


class Roi(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("ny", c_int), ("nx", c_int), ("pitch", c_int), ("dtype", c_int),
                ("ref_id", c_int)]


class CcptError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ccpt error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2310_08770_amd.build.build() first")
        L = ctypes.CDLL(LIB_PATH)
        L.ccpt_default_options.argtypes = [POINTER(Options)]
        L.ccpt_default_options.restype = None
        L.ccpt_create.argtypes = [POINTER(c_void_p), c_int, POINTER(Options)]
        L.ccpt_create.restype = c_int
        L.ccpt_destroy.argtypes = [c_void_p]
        L.ccpt_destroy.restype = None
        L.ccpt_set_reference.argtypes = [c_void_p, POINTER(Image), c_int, c_void_p]
        L.ccpt_set_reference.restype = c_int
        L.ccpt_track_batch.argtypes = [c_void_p, POINTER(Roi), c_int, c_void_p, c_void_p]
        L.ccpt_track_batch.restype = c_int
        L.ccpt_track_batch_static.argtypes = [c_void_p, POINTER(Roi), c_int, c_void_p, c_void_p]
        L.ccpt_track_batch_static.restype = c_int
        L.ccpt_track_grad.argtypes = [c_void_p, POINTER(Roi), c_int, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p]
        L.ccpt_track_grad.restype = c_int
        L.ccpt_fisher.argtypes = [c_void_p, POINTER(Image), c_void_p, c_void_p]
        L.ccpt_fisher.restype = c_int
        L.ccpt_mean_aligned.argtypes = [c_void_p, POINTER(Roi), c_int, c_void_p, c_void_p, c_void_p]
        L.ccpt_mean_aligned.restype = c_int
        L.ccpt_track_update.argtypes = [c_void_p, POINTER(Roi), c_double, c_void_p, c_void_p]
        L.ccpt_track_update.restype = c_int
        L.ccpt_drift_filter.argtypes = [c_void_p, c_int, c_double, c_double, c_void_p, c_void_p]
        L.ccpt_drift_filter.restype = c_int
        L.ccpt_autotune.argtypes = [c_void_p, c_int, c_int, c_void_p]
        L.ccpt_autotune.restype = c_int
        L.ccpt_schedule.argtypes = [c_void_p, c_int, POINTER(c_int), c_int]
        L.ccpt_schedule.restype = c_int
        L.ccpt_get_plan.argtypes = [c_void_p, c_int, c_int, POINTER(Plan)]
        L.ccpt_get_plan.restype = c_int
        L.ccpt_set_plan.argtypes = [c_void_p, c_int, c_int, POINTER(Plan)]
        L.ccpt_set_plan.restype = c_int
        L.ccpt_lanes.argtypes = [c_void_p, POINTER(c_int), c_int]
        L.ccpt_lanes.restype = c_int
        L.ccpt_autotune_batch.argtypes = [c_void_p, POINTER(Roi), c_int, c_void_p]
        L.ccpt_autotune_batch.restype = c_int
        L.ccpt_stage_times.argtypes = [c_void_p, POINTER(c_double), POINTER(c_int), c_int, c_int]
        L.ccpt_stage_times.restype = c_int
        L.ccpt_status_string.argtypes = [c_int]
        L.ccpt_status_string.restype = ctypes.c_char_p
        L.ccpt_last_error.argtypes = [c_void_p, ctypes.c_char_p, c_size_t]
        L.ccpt_last_error.restype = c_int
        _lib = L
    return _lib


EXPORTS = ["ccpt_default_options", "ccpt_create", "ccpt_destroy", "ccpt_set_reference",
           "ccpt_track_batch", "ccpt_track_grad", "ccpt_fisher", "ccpt_autotune", "ccpt_schedule",
           "ccpt_stage_times", "ccpt_status_string", "ccpt_last_error", "ccpt_mean_aligned",
           "ccpt_track_update", "ccpt_drift_filter", "ccpt_track_batch_static", "ccpt_get_plan",
           "ccpt_set_plan", "ccpt_lanes", "ccpt_autotune_batch"]


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype in (torch.uint16, torch.int16):
        return U16
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"frames must be uint16 (or int16 bits), float32 or float64, got {t.dtype}")


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def decode(results: torch.Tensor) -> np.ndarray:
    """Device result buffer -> numpy structured array (RESULT_DTYPE)."""
    raw = results.detach().reshape(-1).to("cpu", torch.uint8).numpy()
    return raw.view(RESULT_DTYPE)


class Tracker:
    """A library context: options, references and workspaces on one GPU."""

    def __init__(self, mode="ccu", eps=200.0, upsample=100, window=1.5, precision="fp32",
                 newton_iters=3, graph=False, profile=False, device=None, streams=1):
        L = lib()
        o = Options()
        L.ccpt_default_options(ctypes.byref(o))
        o.mode = MODES[mode]
        o.eps = float(eps)
        o.upsample = int(upsample)
        o.window = float(window)
        o.precision = PRECISIONS[precision]
        o.newton_iters = int(newton_iters)
        o.flags = ((FLAG_GRAPH if graph else 0) | (FLAG_PROFILE if profile else 0) |
                   (FLAG_STREAMS if streams == 2 else 0))
        self.options = o
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        h = c_void_p()
        rc = L.ccpt_create(ctypes.byref(h), self.device.index, ctypes.byref(o))
        if rc != OK:
            raise CcptError(rc, L.ccpt_status_string(rc).decode())
        self._h = h
        self._refs = []

    def close(self):
        if getattr(self, "_h", None):
            lib().ccpt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            buf = ctypes.create_string_buffer(512)
            lib().ccpt_last_error(self._h, buf, 512)
            raise CcptError(rc, buf.value.decode())

    # ------------------------------------------------------------------
    def set_reference(self, refs, stream=None):
        """refs: one [N, N] tensor or a list of them (device, uint16/float32)."""
        if isinstance(refs, torch.Tensor) and refs.dim() == 2:
            refs = [refs]
        refs = [r.contiguous() for r in refs]
        arr = (Image * len(refs))()
        for i, r in enumerate(refs):
            if r.device != self.device:
                raise ValueError("reference must live on the tracker's device")
            arr[i] = Image(r.data_ptr(), r.shape[0], r.shape[1], r.stride(0), _dtype_code(r))
        self._check(lib().ccpt_set_reference(self._h, arr, len(refs), c_void_p(_stream_handle(stream))))
        self._refs = refs

    def rois(self, frames, ref_ids=None):
        """Roi array for a [n, N, N] tensor or a list of 2-D tensors."""
        if isinstance(frames, torch.Tensor):
            if frames.dim() == 2:
                frames = frames[None]
            if frames.device != self.device:
                raise ValueError("frames must live on the tracker's device")
            if frames.stride(2) != 1:
                raise ValueError("frame rows must be contiguous")
            n, ny, nx = frames.shape
            ids = [0] * n if ref_ids is None else ref_ids
            base, step, es = frames.data_ptr(), frames.stride(0), frames.element_size()
            pitch, code = frames.stride(1), _dtype_code(frames)
            arr = (Roi * n)()
            for i in range(n):
                arr[i] = Roi(base + i * step * es, ny, nx, pitch, code, int(ids[i]))
            return arr, n
        else:
            seq = list(frames)
        n = len(seq)
        if ref_ids is None:
            ref_ids = [0] * n
        arr = (Roi * n)()
        for i, f in enumerate(seq):
            if f.device != self.device:
                raise ValueError("frames must live on the tracker's device")
            if f.stride(1) != 1:
                raise ValueError("frame rows must be contiguous")
            arr[i] = Roi(f.data_ptr(), f.shape[0], f.shape[1], f.stride(0), _dtype_code(f), int(ref_ids[i]))
        return arr, n

    def track(self, frames, ref_ids=None, out=None, stream=None, rois=None):
        """Tracks frames; returns the device result buffer (uint8 [n, 72]).
        Use decode() for a numpy view.  `rois` reuses a prepared roi array."""
        if rois is None:
            rois = self.rois(frames, ref_ids)
        arr, n = rois
        if out is None:
            out = torch.empty((n, RESULT_BYTES), dtype=torch.uint8, device=self.device)
        self._check(lib().ccpt_track_batch(self._h, arr, n, c_void_p(out.data_ptr()),
                                           c_void_p(_stream_handle(stream))))
        return out

    def track_static(self, frames=None, ref_ids=None, out=None, stream=None, rois=None):
        """track() through ccpt_track_batch_static: no device allocation by
        the library (its static scratch holds every per-call buffer); `out`
        must then be supplied by the caller as well."""
        if rois is None:
            rois = self.rois(frames, ref_ids)
        arr, n = rois
        if out is None:
            raise ValueError("track_static needs a preallocated out buffer [n, 72] uint8")
        self._check(lib().ccpt_track_batch_static(self._h, arr, n, c_void_p(out.data_ptr()),
                                                  c_void_p(_stream_handle(stream))))
        return out

    def track_grad(self, frames, fwd, g_d, g_peak=None, want_frames=True, want_ref=True,
                   ref_ids=None, stream=None):
        """Backward of track() for L = sum g_d . d + g_peak * C(d)."""
        arr, n = self.rois(frames, ref_ids)
        g_d = g_d.to(self.device, torch.float64).contiguous()
        gp = g_peak.to(self.device, torch.float64).contiguous() if g_peak is not None else None
        gf = gr = None
        if want_frames:
            total = sum(arr[i].ny * arr[i].nx for i in range(n))
            gf = torch.empty(total, dtype=torch.float32, device=self.device)
        if want_ref:
            total = sum(r.shape[0] * r.shape[1] for r in self._refs)
            gr = torch.empty(total, dtype=torch.float32, device=self.device)
        self._check(lib().ccpt_track_grad(
            self._h, arr, n, c_void_p(fwd.data_ptr()), c_void_p(g_d.data_ptr()),
            c_void_p(gp.data_ptr() if gp is not None else 0),
            c_void_p(gf.data_ptr() if gf is not None else 0),
            c_void_p(gr.data_ptr() if gr is not None else 0),
            c_void_p(_stream_handle(stream))))
        return gf, gr

    def fisher(self, mu, stream=None):
        """Fisher matrix (2x2, float64 device tensor) of the displacement for
        an expected image mu under Poisson noise."""
        mu = mu.contiguous()
        img = Image(mu.data_ptr(), mu.shape[0], mu.shape[1], mu.stride(0), _dtype_code(mu))
        out = torch.empty(3, dtype=torch.float64, device=self.device)
        self._check(lib().ccpt_fisher(self._h, ctypes.byref(img), c_void_p(out.data_ptr()),
                                      c_void_p(_stream_handle(stream))))
        f = out
        return torch.stack([torch.stack([f[0], f[1]]), torch.stack([f[1], f[2]])])

    def mean_aligned(self, frames, fwd, stream=None):
        """Offline reference of Eq. (8): the mean of the frames shifted back by
        their displacements in fwd (track() results for the same frames, in
        order), as an [N, N] float32 device tensor."""
        arr, n = self.rois(frames)
        N = arr[0].nx
        out = torch.empty((N, N), dtype=torch.float32, device=self.device)
        self._check(lib().ccpt_mean_aligned(self._h, arr, n, c_void_p(fwd.data_ptr()),
                                            c_void_p(out.data_ptr()), c_void_p(_stream_handle(stream))))
        return out

    def track_update(self, frame, a0, out=None, ref_id=0, stream=None):
        """Real-time tracking of one frame with the reference low-pass of
        Eq. (9); returns the device result buffer (uint8 [1, 72])."""
        arr, n = self.rois(frame, [ref_id])
        if n != 1:
            raise ValueError("one frame per call")
        if out is None:
            out = torch.empty((1, RESULT_BYTES), dtype=torch.uint8, device=self.device)
        self._check(lib().ccpt_track_update(self._h, arr, float(a0), c_void_p(out.data_ptr()),
                                            c_void_p(_stream_handle(stream))))
        return out

    def stage_times(self, reset=True):
        """{stage: (total ms, launches)} recorded with profile=True."""
        k = len(STAGES)
        ms = (c_double * k)()
        cnt = (c_int * k)()
        self._check(lib().ccpt_stage_times(self._h, ms, cnt, k, 1 if reset else 0))
        return {STAGES[i]: (ms[i], cnt[i]) for i in range(k)}

    def autotune(self, n, batch, stream=None, cache=None):
        """Tunes the chunk size for n x n frames in batches of `batch` (needs a
        reference of that size).  With `cache` (a JSON file path) the choice is
        read from / written to it, keyed by GPU arch, size, u, precision, mode."""
        key = None
        if cache:
            import json
            props = torch.cuda.get_device_properties(self.device)
            arch = getattr(props, "gcnArchName", props.name)
            o = self.options
            key = f"{arch}|N={n}|batch={batch}|u={o.upsample}|prec={o.precision}|mode={o.mode}"
            try:
                with open(cache) as fh:
                    table = json.load(fh)
            except (OSError, ValueError):
                table = {}
            if key in table:
                self.set_chunk(n, int(table[key]))
                return int(table[key])
        self._check(lib().ccpt_autotune(self._h, int(n), int(batch), c_void_p(_stream_handle(stream))))
        chunk = self.chunk(n)
        if cache:
            table[key] = chunk
            with open(cache, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
        return chunk

    def chunk(self, n):
        """Frames per launch chunk currently used for n x n frames."""
        c = c_int(0)
        self._check(lib().ccpt_schedule(self._h, int(n), ctypes.byref(c), 0))
        return c.value

    def set_chunk(self, n, chunk):
        c = c_int(int(chunk))
        self._check(lib().ccpt_schedule(self._h, int(n), ctypes.byref(c), 1))

    def plan(self, ny, nx=None):
        """Launch plan in force for ny x nx frames: dict(chunk, split_blocks, fused_min)."""
        p = Plan()
        self._check(lib().ccpt_get_plan(self._h, int(ny), int(ny if nx is None else nx), ctypes.byref(p)))
        return dict(chunk=p.chunk, split_blocks=p.split_blocks, fused_min=p.fused_min)

    def set_plan(self, ny, nx=None, chunk=0, split_blocks=-1, fused_min=-1):
        """Sets the launch plan of ny x nx frames (0 / -1 fields: defaults)."""
        p = Plan(int(chunk), int(split_blocks), int(fused_min))
        self._check(lib().ccpt_set_plan(self._h, int(ny), int(ny if nx is None else nx), ctypes.byref(p)))

    def lanes(self, set_to=None):
        """Most concurrent size-group lanes a call uses (reads, or sets when set_to is given)."""
        if set_to is not None:
            c = c_int(int(set_to))
            self._check(lib().ccpt_lanes(self._h, ctypes.byref(c), 1))
        c = c_int(0)
        self._check(lib().ccpt_lanes(self._h, ctypes.byref(c), 0))
        return c.value

    def autotune_batch(self, frames=None, ref_ids=None, rois=None, stream=None):
        """Tunes lanes and every shape's launch plan by timing this batch itself."""
        if rois is None:
            rois = self.rois(frames, ref_ids)
        arr, n = rois
        self._check(lib().ccpt_autotune_batch(self._h, arr, n, c_void_p(_stream_handle(stream))))


def drift_filter(r, a0, rate_limit=0.0, state=None):
    """Drift correction of Eq. (10)-(12) on displacements r ([n, 2], host):
    returns (r - R, state); pass the returned state to continue a stream."""
    r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1, 2)
    out = np.empty_like(r)
    st = np.zeros(3) if state is None else np.array(state, dtype=np.float64).reshape(3)
    rc = lib().ccpt_drift_filter(r.ctypes.data, r.shape[0], float(a0), float(rate_limit),
                                 st.ctypes.data, out.ctypes.data)
    if rc != OK:
        raise CcptError(rc, "ccpt_drift_filter: bad arguments")
    return out, st
