"""Continuous-batching request loop over the cipher library.

Encrypt and decrypt requests for many video streams arrive at their own
times.  The loop keeps the key state and scratch resident on the device (one
sender context for encrypt requests, one receiver context for decrypt
requests), and whenever fewer than ``max_inflight`` batches of a kind are on
the GPU it launches the next batch from the requests that have arrived:

* admission in arrival order, by device-memory footprint: a request holds
  its input, its output and its per-frame scratch while in flight, and the
  sum over in-flight requests stays within ``hbm_budget`` (a request larger
  than the whole budget is admitted alone);
* per-stream order: a stream's frame t+1 is never launched before frame t
  (the chain of the paper's Alg. 1 is serial per stream), and frames of one
  stream in one batch go in sequence order;
* with ``hash_first``, an encrypt request's frame hash (SHA-256, the longest
  serial part, and independent of the stream's previous frame) is launched
  as soon as the request arrives, in "hash" batches that ignore stream
  order; only the key chain, keystream and confusion wait for the
  stream's previous frame (encrypt_frames_hashed);
* a batch is one library call (encrypt_frames or decrypt_frames) over any
  mix of streams; with a ``batch_class`` (e.g. the resolution) only
  requests of one class share a batch, so small frames do not wait for the
  serial SHA-256 and key schedule of large ones; consecutive batches of a
  kind go to rotating device streams, so they overlap on the device and a
  batch's key chain runs while earlier batches' keygen and confusion
  finish.

The scheduling core (:class:`Scheduler`) is plain Python over an abstract
backend, so that its admission and ordering rules are testable on the CPU;
:class:`GpuBackend` runs batches through the C ABI.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple


@dataclasses.dataclass
class Request:
    """One frame to encrypt (kind "enc") or decrypt (kind "dec")."""
    stream: int
    seq: int
    kind: str
    frame: object                 # device uint8 (h, w, 3)
    out: object                   # device uint8 (h, w, 3), written by the batch
    hashes: object = None         # device uint8 (32,): output for "enc", input for "dec"
    nbytes: int = 0               # device footprint while in flight
    arrival: float = 0.0          # host time the request became available
    launched: float = float("nan")
    done: float = float("nan")
    admitted: bool = False        # holds its footprint (from its first launch until done)
    hashed: bool = False          # "enc" with hash_first: its SHA-256 stage has completed

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Scheduler:
    """Admission, ordering and batching.  ``launch(kind, requests)`` starts
    a batch and returns a handle with ``query() -> bool`` (True once the
    batch has completed).  At most ``max_inflight`` batches of a kind (of a
    kind and class, with ``batch_class``) are in flight."""

    def __init__(self, launch: Callable[[str, List[Request]], object], hbm_budget: int, max_inflight=2,
                 max_batch: int = 512, clock: Callable[[], float] = time.perf_counter,
                 batch_class: Optional[Callable[[Request], object]] = None, max_stream_inflight: int = 0,
                 hash_first: bool = False):
        self.launch = launch
        # encrypt requests go through a "hash" batch first (see the module notes)
        self.hash_first = hash_first
        # max_inflight: an int, or a function (kind, class) -> int
        self.max_inflight = max_inflight if callable(max_inflight) else (lambda kind, cls, m=max_inflight: m)
        # at most this many frames of one stream in flight (0 = no limit), e.g.
        # to bound a per-stream ring of output buffers
        self.max_stream_inflight = max_stream_inflight
        self.stream_inflight: Dict[Tuple[str, int], int] = collections.defaultdict(int)
        # Requests of different classes (e.g. resolutions) never share a
        # batch, so a batch's completion is not held back by slower frames.
        self.batch_class = batch_class
        self.hbm_budget = hbm_budget
        self.max_batch = max_batch
        self.clock = clock
        self.pending: Dict[str, Deque[Request]] = {k: collections.deque() for k in ("hash", "enc", "dec")}
        self.inflight: List[Tuple[str, object, List[Request]]] = []
        self.inflight_bytes = 0
        self.next_seq: Dict[Tuple[str, int], int] = collections.defaultdict(int)  # next seq to launch
        # next seq to admit: admission is in stream order too, so the frames a
        # stream holds are always a prefix and its oldest one can proceed
        self.next_admit: Dict[Tuple[str, int], int] = collections.defaultdict(int)
        self.completed: List[Request] = []
        self.batches: List[Tuple[str, int]] = []  # (kind, size) of every launched batch

    def submit(self, req: Request) -> None:
        self.pending["hash" if self.hash_first and req.kind == "enc" else req.kind].append(req)

    def _class_of(self, r: Request):
        return self.batch_class(r) if self.batch_class else None

    def _inflight_of(self, kind: str, cls=None) -> int:
        """Batches of a kind (and class, with batch classes) on the GPU."""
        return sum(1 for k, _, reqs in self.inflight if k == kind and self._class_of(reqs[0]) == cls)

    def retire(self) -> int:
        """Record completion of finished batches; returns how many retired."""
        keep, n = [], 0
        for kind, handle, reqs in self.inflight:
            if handle.query():
                t = self.clock()
                if kind == "hash":
                    # on to the ordered stage; the footprint stays held
                    for r in reqs:
                        r.hashed = True
                    self.pending["enc"].extend(reqs)
                else:
                    for r in reqs:
                        r.done = t
                        self.inflight_bytes -= r.nbytes
                        self.stream_inflight[(r.kind, r.stream)] -= 1
                    self.completed.extend(reqs)
                n += 1
            else:
                keep.append((kind, handle, reqs))
        self.inflight = keep
        return n

    def _form_batch(self, kind: str) -> List[Request]:
        """Requests to launch now, in arrival order: each the next frame of its
        stream to admit and (except in "hash" batches) to launch, counting
        frames taken earlier in this batch, within the memory budget
        (charged once, at a request's first launch).  Passes over the queue repeat while they take
        something, so a frame that arrived before its predecessor goes in
        the same batch as it."""
        q = self.pending[kind]
        batch: List[Request] = []
        cls = None
        expect: Dict[Tuple[str, int], int] = {}
        admitted_now: Dict[Tuple[str, int], int] = {}
        budget = self.hbm_budget - self.inflight_bytes
        full = False
        rest = list(q)
        progress = True
        while progress and not full:
            progress = False
            left: List[Request] = []
            for i, r in enumerate(rest):
                key = (r.kind, r.stream)
                ordered = kind != "hash"     # a hash may run beside its predecessor's later stage
                want = expect.get(key, self.next_seq[key])
                rc = self._class_of(r)
                taken = admitted_now.get(key, 0)   # frames of this stream admitted by this batch
                if full or (ordered and r.seq != want) or (batch and rc != cls) or \
                        (not r.admitted and r.seq != self.next_admit[key] + taken) or \
                        (not batch and self._inflight_of(kind, rc) >= self.max_inflight(kind, rc)) or \
                        (not r.admitted and self.max_stream_inflight and
                         self.stream_inflight[key] + taken >= self.max_stream_inflight):
                    left.append(r)
                    continue
                if not r.admitted:
                    alone = not batch and self.inflight_bytes == 0
                    if r.nbytes > budget and not alone:
                        full = True     # admission stops at the first request that does not fit
                        left.append(r)
                        continue
                    budget -= r.nbytes
                    admitted_now[key] = taken + 1
                batch.append(r)
                cls = rc
                if ordered:
                    expect[key] = want + 1
                progress = True
                if len(batch) >= self.max_batch:
                    full = True
            rest = left
        q.clear()
        q.extend(rest)
        return batch

    def pump(self) -> int:
        """Retire finished batches and launch new ones while slots are free.
        Returns the number of batches launched."""
        self.retire()
        launched = 0
        for kind in ("enc", "dec", "hash"):
            while self.pending[kind]:
                batch = self._form_batch(kind)
                if not batch:
                    break
                t = self.clock()
                for r in batch:
                    if not r.admitted:
                        r.admitted = True
                        r.launched = t
                        self.inflight_bytes += r.nbytes
                        self.stream_inflight[(r.kind, r.stream)] += 1
                        self.next_admit[(r.kind, r.stream)] = r.seq + 1
                    if kind != "hash":
                        self.next_seq[(kind, r.stream)] = r.seq + 1
                handle = self.launch(kind, batch)
                self.inflight.append((kind, handle, batch))
                self.batches.append((kind, len(batch)))
                launched += 1
        return launched

    def idle(self) -> bool:
        return not self.inflight and not any(self.pending.values())


class _HipStream:
    """A HIP stream of its own (non-blocking), for torch as an ExternalStream.

    torch.cuda.Stream() hands out streams from a pool of 32 that torch creates
    all at once; HIP maps streams onto a fixed number of hardware queues
    (GPU_MAX_HW_QUEUES), so with the pool present the library's own streams
    would share queues with active device streams and wait behind their
    work.  Streams created one by one take the next free queue.

    The streams are never destroyed: torch may still record or query events
    on a stream after its user is done with it (tensors whose use was
    recorded on it, completion events), so a closed backend returns its
    streams to a process-wide pool and the next one reuses them."""

    _hip = None
    _free: List["_HipStream"] = []

    def __init__(self, torch):
        import ctypes
        if _HipStream._hip is None:
            _HipStream._hip = ctypes.CDLL("libamdhip64.so")
            _HipStream._hip.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        self.ptr = ctypes.c_void_p()
        rc = _HipStream._hip.hipStreamCreateWithFlags(ctypes.byref(self.ptr), 1)   # hipStreamNonBlocking
        if rc != 0:
            raise RuntimeError(f"hipStreamCreateWithFlags failed ({rc})")
        self.stream = torch.cuda.ExternalStream(self.ptr.value)

    @classmethod
    def take(cls, torch) -> "_HipStream":
        return cls._free.pop() if cls._free else cls(torch)

    def release(self) -> None:
        self.stream.synchronize()
        _HipStream._free.append(self)


class GpuBackend:
    """Runs batches through the library.  Encrypt requests go to sender
    contexts and decrypt requests to receiver contexts; with
    ``batch_class`` there is one context pair per class (each stream's frames
    always fall in one class, so each chain lives in one context), so that
    batches of different classes never queue behind each other on a
    context's streams.  Each (kind, class) rotates over ``device_streams``
    device streams.  ``overlap`` (parts, side streams, scratch slots; or a
    function (kind, class) -> that) configures each context."""

    def __init__(self, key32: bytes, gamma: float, n: int, max_streams: int, scratch_bytes: int,
                 overlap=None, device_streams=2,
                 classes: Optional[Sequence[object]] = None,
                 batch_class: Optional[Callable[[Request], object]] = None, hash_first: bool = False):
        import torch

        from . import vcipher as V
        self.torch = torch
        self.V = V
        self.n = n
        self.batch_class = batch_class
        self.launch_seconds = 0.0   # host time spent enqueueing batches
        self.ctx: Dict[Tuple[str, object], object] = {}
        self.streams: Dict[Tuple[str, object], list] = {}
        self.turn: Dict[Tuple[str, object], int] = {}
        for cls in (classes if classes else [None]):
            for kind in ("enc", "dec"):
                c = V.Cipher.from_bytes(key32, gamma, n, max_streams=max_streams, scratch_bytes=scratch_bytes)
                ov = overlap(kind, cls) if callable(overlap) else overlap
                if ov:
                    c.overlap(*ov)
                self.ctx[(kind, cls)] = c
                ns = device_streams(kind, cls) if callable(device_streams) else device_streams
                self.streams[(kind, cls)] = [_HipStream.take(torch) for _ in range(ns)]
                self.turn[(kind, cls)] = 0
            if hash_first:
                # "hash" batches run on the sender context of the class
                ns = device_streams("hash", cls) if callable(device_streams) else device_streams
                self.streams[("hash", cls)] = [_HipStream.take(torch) for _ in range(ns)]
                self.turn[("hash", cls)] = 0

    def footprint(self, w: int, h: int) -> int:
        """Device bytes a request holds while in flight: input, output and scratch."""
        return 2 * 3 * w * h + self.V.vc_scratch_per_frame(w, h, self.n)

    def status_ok(self) -> bool:
        return all(c.status() == 0 for c in self.ctx.values())

    def launch(self, kind: str, reqs: Sequence[Request]):
        t0 = time.perf_counter()
        torch, V = self.torch, self.V
        key = (kind, self.batch_class(reqs[0]) if self.batch_class else None)
        st = self.streams[key][self.turn[key]].stream
        self.turn[key] = (self.turn[key] + 1) % len(self.streams[key])
        c = self.ctx[("enc", key[1]) if kind == "hash" else key]
        frames = [r.frame for r in reqs]
        outs = [r.out for r in reqs]
        streams = [r.stream for r in reqs]
        seqs = [r.seq for r in reqs]
        hashes = torch.empty((len(reqs), 32), dtype=torch.uint8, device=frames[0].device)
        with torch.cuda.stream(st):
            if kind == "hash":
                V.vc_hash_frames(c.ctx, frames, hashes, st)
                for i, r in enumerate(reqs):
                    r.hashes.copy_(hashes[i])
            elif kind == "dec" or reqs[0].hashed:
                for i, r in enumerate(reqs):
                    hashes[i].copy_(r.hashes)
                fn = V.decrypt_frames if kind == "dec" else V.encrypt_frames_hashed
                fn(c.ctx, frames, streams, seqs, hashes, outs, st)
            else:
                V.encrypt_frames(c.ctx, frames, streams, seqs, hashes, outs, st)
                for i, r in enumerate(reqs):
                    if r.hashes is not None:
                        r.hashes.copy_(hashes[i])
            ev = torch.cuda.Event()
            ev.record(st)
        hashes.record_stream(st)
        self.launch_seconds += time.perf_counter() - t0
        return ev

    def reset_chains(self, streams: Sequence[int]) -> None:
        """Back to the key for the given streams in every context (e.g. after a
        warm-up that ran frames through them).  Call with the device idle."""
        for c in self.ctx.values():
            for s in streams:
                c.reset(s)

    def close(self) -> None:
        for c in self.ctx.values():
            c.close()
        for ss in self.streams.values():
            for st in ss:
                st.release()
        self.ctx.clear()
        self.streams.clear()
