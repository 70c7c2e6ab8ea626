"""Python face of the library: torch supplies device memory and the current
stream, the HIP kernels behind the C ABI do all of the completion.

    out = complete(depth)                  # 2-D float32 tensor on the GPU
    outs = complete_batch([d0, d1, ...])   # frames of any sizes, one launch per phase
"""
from __future__ import annotations

import array
import atexit
import ctypes
import dataclasses
import warnings
from typing import List, Optional, Sequence

import torch

from . import _lib as L

SE_FULL, SE_CROSS, SE_DIAMOND, SE_CIRCLE = 0, 1, 2, 3
BLUR_GAUSSIAN, BLUR_BILATERAL = 0, 1
N_STAGES = 9


@dataclasses.dataclass
class Params:
    """Mirror of ipb_params; defaults are the paper's final design
    (Sec. III; Tables 2 and 3)."""
    dilate_shape: int = SE_DIAMOND
    dilate_size: int = 5
    close_size: int = 5
    fill_size: int = 7
    extrapolate: int = 1
    large_fill_size: int = 31
    median_size: int = 5
    gauss_size: int = 5
    gauss_sigma: float = 0.0
    max_depth: float = 100.0
    valid_thresh: float = 0.1
    tile_local: int = 0
    tile_global: int = 0
    blur: int = BLUR_GAUSSIAN            # stage 8: Gaussian, or bilateral (Sec. IV, Table 3)
    bilateral_sigma_space: float = 2.0
    bilateral_sigma_color: float = 1.5
    extend_rows: int = 0                 # stage-5 reach above a column's top; 0 = to row 0

    def to_c(self) -> L.CParams:
        """A fresh ipb_params for these values (the caller may change it)."""
        key = tuple(self.__dict__.values())
        c = _C_PARAMS.get(key)
        if c is None:
            c = L.CParams()
            L.lib().ipb_params_default(ctypes.byref(c))
            for f in dataclasses.fields(self):
                setattr(c, f.name, getattr(self, f.name))
            if len(_C_PARAMS) >= 256:
                _C_PARAMS.clear()
            _C_PARAMS[key] = c
        return L.CParams.from_buffer_copy(c)


# converted parameter sets by field values (a per-call conversion costs a
# few microseconds, a sizeable share of one small frame's host time)
_C_PARAMS: dict = {}


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _launch_stream(stream: Optional[torch.cuda.Stream], device: torch.device):
    """The stream the call runs on and whether it is another than the
    current one (then buffers the call takes from torch's allocator are
    allocated under it, and tensors from the current stream are recorded on
    it, so that torch's caching allocator does not hand their memory to other
    work while the kernels still use it)."""
    cur = torch.cuda.current_stream(device)
    if stream is None or stream == cur:
        return cur, False
    return stream, True


# streams with hardware queues of their own, per device index, made on
# first request and kept until the interpreter exits
_QUEUE_STREAMS: dict = {}


def _release_queue_streams() -> None:
    # at interpreter exit, ahead of the runtime's own teardown (and of a
    # profiler's, which has ended in a fault over streams still alive then)
    lib = L.lib()
    for idx, streams in list(_QUEUE_STREAMS.items()):
        try:
            with torch.cuda.device(idx):
                torch.cuda.synchronize()
                for s in streams:
                    if isinstance(s, torch.cuda.ExternalStream):
                        lib.ipb_stream_destroy(ctypes.c_void_p(s.cuda_stream))
        except RuntimeError:
            pass        # a device already in error: the runtime's teardown takes them
    _QUEUE_STREAMS.clear()


def queue_streams(n: int, device=None) -> List[torch.cuda.Stream]:
    """`n` streams of `device` (default: the current one), each on a
    hardware queue of its own (ipb_stream_create), for batches kept in
    flight side by side.  Streams from torch's pool share the runtime's few
    hardware queues, at times two of them one queue, and batches on a
    shared queue run one after the other.  The streams are made once per
    device and live until the interpreter exits; every caller that asks for `n`
    gets the first `n` of them, so independent users of one process share
    them.  They synchronise with the legacy null stream, as any stream
    created without flags does.  Should the runtime refuse such a stream,
    a warning says so and torch's pool streams stand in."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    if not _QUEUE_STREAMS:
        atexit.register(_release_queue_streams)
    have = _QUEUE_STREAMS.setdefault(idx, [])
    lib = L.lib()
    with torch.cuda.device(idx):
        while len(have) < n:
            h = ctypes.c_void_p()
            st = lib.ipb_stream_create(ctypes.byref(h))
            if st == L.IPB_ERR_HIP:
                # a runtime that refuses compute-unit masks: torch's pool
                # streams, which may share hardware queues
                warnings.warn(f"ipb_stream_create: {L.status_string(st)} (hipError "
                              f"{lib.ipb_last_hip_error()}); using torch's pool streams", RuntimeWarning)
                have.append(torch.cuda.Stream(device=torch.device("cuda", idx)))
                continue
            L.check(st, "ipb_stream_create")
            have.append(torch.cuda.ExternalStream(h.value, device=torch.device("cuda", idx)))
    return have[:n]


def _record(stream: torch.cuda.Stream, *tensors: torch.Tensor) -> None:
    for t in tensors:
        t.record_stream(stream)


def _check_map(t: torch.Tensor, name: str) -> None:
    if not isinstance(t, torch.Tensor) or t.dim() != 2:
        raise ValueError(f"{name} must be a 2-D tensor")
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor on the GPU")


def _workspace(nbytes: int, device: torch.device) -> torch.Tensor:
    # 256-byte aligned device workspace from torch's allocator
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    shift = (-buf.data_ptr()) % 256
    return buf[shift:shift + nbytes]


def workspace_bytes(H: int, W: int, params: Optional[Params] = None) -> int:
    p = (params or Params()).to_c()
    return int(L.lib().ipb_workspace_bytes(H, W, ctypes.byref(p)))


def complete(depth: torch.Tensor, params: Optional[Params] = None, out: Optional[torch.Tensor] = None,
             stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Dense map of one sparse H x W depth map (ipb_complete_ws)."""
    return complete_stage(depth, N_STAGES, params, out, stream)


def complete_stage(depth: torch.Tensor, last_stage: int, params: Optional[Params] = None,
                   out: Optional[torch.Tensor] = None,
                   stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Map after stage `last_stage` (1..9; stages 1-8 in the inverted domain).

    Runs on `stream` (default: the current stream); the caller orders that
    stream after whatever produced `depth`.  With another stream than the
    current one, the workspace and a default `out` are allocated under
    `stream`, and `depth` and a given `out` are recorded on it."""
    _check_map(depth, "depth")
    H, W = depth.shape
    s, other = _launch_stream(stream, depth.device)
    p = (params or Params()).to_c()
    nb = int(L.lib().ipb_workspace_bytes(H, W, ctypes.byref(p)))
    if nb == 0:
        L.check(L.IPB_ERR_INVALID_ARG, "ipb_workspace_bytes")
    if other:
        if out is not None:
            _check_map(out, "out")
            _record(s, out)
        _record(s, depth)
        with torch.cuda.stream(s):
            if out is None:
                out = torch.empty_like(depth)
            ws = _workspace(nb, depth.device)
    else:
        if out is None:
            out = torch.empty_like(depth)
        ws = _workspace(nb, depth.device)
    _check_map(out, "out")
    st = L.lib().ipb_complete_stage(ctypes.c_void_p(depth.data_ptr()), H, W, ctypes.byref(p),
                                    ctypes.c_void_p(out.data_ptr()), last_stage,
                                    ctypes.c_void_p(ws.data_ptr()), nb, ctypes.c_void_p(s.cuda_stream))
    L.check(st, "ipb_complete_stage")
    return out


def complete_alloc(depth: torch.Tensor, params: Optional[Params] = None, out: Optional[torch.Tensor] = None,
                   stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """As complete(), with the library's own stream-ordered workspace
    (ipb_complete)."""
    _check_map(depth, "depth")
    H, W = depth.shape
    s, other = _launch_stream(stream, depth.device)
    if other:
        if out is not None:
            _check_map(out, "out")
            _record(s, out)
        _record(s, depth)
        with torch.cuda.stream(s):
            if out is None:
                out = torch.empty_like(depth)
    elif out is None:
        out = torch.empty_like(depth)
    _check_map(out, "out")
    p = (params or Params()).to_c()
    st = L.lib().ipb_complete(ctypes.c_void_p(depth.data_ptr()), H, W, ctypes.byref(p),
                              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    L.check(st, "ipb_complete")
    return out


def _is_map(t) -> bool:
    return (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.dim() == 2
            and t.is_contiguous())


def _frames_array(ins: Sequence[torch.Tensor], outs: Sequence[torch.Tensor]):
    """The ipb_frame array of a batch and its frames' shortest side.  The
    array is written in one copy from a flat list (input pointer, output
    pointer, H | W << 32 per frame, the struct's layout): a batch of 64
    frames is marshalled on the host before every graph replay, and setting
    the struct fields one by one cost several microseconds per frame."""
    n = len(ins)
    if len(outs) != n:
        raise ValueError(f"{n} frames but {len(outs)} outputs")
    vals = []
    side = 1 << 30
    for i in range(n):
        a, b = ins[i], outs[i]
        if not _is_map(a):
            _check_map(a, f"frames[{i}]")
        if not _is_map(b):
            _check_map(b, f"outs[{i}]")
        H, W = a.shape
        if b.shape != a.shape:
            raise ValueError(f"frame {i}: output shape differs from input")
        vals += (a.data_ptr(), b.data_ptr(), H | (W << 32))
        side = min(side, H, W)
    return (L.CFrame * n).from_buffer_copy(array.array("q", vals)), side


def frames_array(ins: Sequence[torch.Tensor], outs: Sequence[torch.Tensor]):
    """The ipb_frame array of a batch (inputs and outputs checked)."""
    return _frames_array(ins, outs)[0]


def batch_workspace_bytes(frames: Sequence[torch.Tensor], params: Optional[Params] = None,
                          outs: Optional[Sequence[torch.Tensor]] = None) -> int:
    outs = list(outs) if outs is not None else list(frames)
    arr = frames_array(frames, outs)
    p = (params or Params()).to_c()
    return int(L.lib().ipb_batch_workspace_bytes(arr, len(frames), ctypes.byref(p)))


def complete_batch(frames: Sequence[torch.Tensor], params: Optional[Params] = None,
                   outs: Optional[Sequence[torch.Tensor]] = None,
                   stream: Optional[torch.cuda.Stream] = None) -> List[torch.Tensor]:
    """Complete frames of any sizes together (ipb_complete_batch).  Stream
    rules as complete_stage()."""
    frames = list(frames)
    if not frames:
        return []
    dev = frames[0].device
    s, other = _launch_stream(stream, dev)
    if other:
        _record(s, *frames)
        if outs is not None:
            _record(s, *outs)
    with torch.cuda.stream(s):
        outs = list(outs) if outs is not None else [torch.empty_like(f) for f in frames]
        arr = frames_array(frames, outs)
        p = (params or Params()).to_c()
        nb = int(L.lib().ipb_batch_workspace_bytes(arr, len(frames), ctypes.byref(p)))
        if nb == 0:
            L.check(L.IPB_ERR_INVALID_ARG, "ipb_batch_workspace_bytes")
        ws = _workspace(nb, dev)
    st = L.lib().ipb_complete_batch(arr, len(frames), ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()), nb,
                                    ctypes.c_void_p(s.cuda_stream))
    L.check(st, "ipb_complete_batch")
    return outs
