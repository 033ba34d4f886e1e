"""Continuous batching of per-frame requests: Python side of the library's
native serving core (include/vcipher.h, "Serving").

Encrypt and decrypt requests for many video streams arrive at their own
times.  The scheduling rules live in the library (vc_sched, vc_server):

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
* a batch is one library call over any mix of streams of one class (the
  server uses the resolution, so small frames do not wait for the serial
  SHA-256 and key schedule of large ones), launched whenever fewer than
  ``max_inflight`` batches of its kind and class are in flight
  (``max_inflight_hash`` for hash batches, 0 = the same).

:class:`Scheduler` drives the native core with a backend written in Python
(the CPU tests use fake backends); :class:`Server` is the native core with
its own GPU backend: contexts, device streams and completion events, and a
native trace-replay loop (:meth:`Server.run_trace`).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import sys
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from . import vcipher as V

KINDS = ("enc", "dec", "hash")


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
    hashed: bool = False          # "enc" with hash_first: went through a hash batch
    status: int = 0               # VC_OK, a failed launch's status, or VC_EORDER behind one

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Scheduler:
    """The library's scheduling core (vc_sched) over a backend in Python:
    ``launch(kind, requests)`` starts a batch (kind "enc", "dec" or "hash")
    and returns a handle with ``query() -> bool`` (True once the batch has
    completed).  ``batch_class(request)`` (optional) gives the class of a
    request; requests of different classes never share a batch."""

    def __init__(self, launch: Callable[[str, List[Request]], object], hbm_budget: int, max_inflight: int = 2,
                 max_batch: int = 512, clock: Callable[[], float] = time.perf_counter,
                 batch_class: Optional[Callable[[Request], object]] = None, max_stream_inflight: int = 0,
                 hash_first: bool = False, max_inflight_hash: int = 0):
        self.launch = launch
        self.clock = clock
        self.batch_class = batch_class
        cfg = V.VcSchedConfig(int(hbm_budget), int(max_inflight), int(max_batch), int(max_stream_inflight),
                              1 if hash_first else 0, int(max_inflight_hash), 0)
        h = C.c_void_p()
        V._check(V.lib.vc_sched_create(C.byref(cfg), C.byref(h)), "vc_sched_create")
        self._h = h.value
        self._reqs: Dict[int, Request] = {}
        self._classes: Dict[object, int] = {}
        self._handles: Dict[int, object] = {}
        self._next_tag = 0
        self._next_handle = 0
        self._now = 0.0
        self._error = None
        self.completed: List[Request] = []
        self.batches: List[Tuple[str, int]] = []  # (kind, size) of every launched batch
        # the callbacks must outlive every pump
        self._launch_cb = V.LAUNCH_FN(self._on_launch)
        self._query_cb = V.QUERY_FN(self._on_query)

    def close(self) -> None:
        if self._h:
            V.lib.vc_sched_destroy(C.c_void_p(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, r: Request) -> None:
        tag = self._next_tag
        self._next_tag += 1
        self._reqs[tag] = r
        cls = 0
        if self.batch_class is not None:
            cls = self._classes.setdefault(self.batch_class(r), len(self._classes) + 1)
        req = V.VcRequest(tag=tag, kind=0 if r.kind == "enc" else 1, stream=r.stream, seq=r.seq, cls=cls,
                          nbytes=int(r.nbytes), arrival=float(r.arrival))
        V._check(V.lib.vc_sched_submit(C.c_void_p(self._h), C.byref(req)), "vc_sched_submit")

    def _on_launch(self, _user, kind, count, tags):
        try:
            reqs = [self._reqs[tags[i]] for i in range(count)]
            for r in reqs:
                if r.launched != r.launched:      # first launch
                    r.launched = self._now
            handle = self.launch(KINDS[kind], reqs)
            hid = self._next_handle
            self._next_handle += 1
            self._handles[hid] = handle
            self.batches.append((KINDS[kind], count))
            return hid
        except Exception:
            self._error = sys.exc_info()
            return V.VC_EDEVICE

    def _on_query(self, _user, hid):
        try:
            if self._handles[hid].query():
                del self._handles[hid]
                return 1
            return 0
        except Exception:
            self._error = sys.exc_info()
            return V.VC_EDEVICE

    def pump(self) -> int:
        """Retire finished batches and launch new ones while slots are free.
        Returns the number of batches launched."""
        self._now = self.clock()
        n = V.lib.vc_sched_pump(C.c_void_p(self._h), self._now, self._launch_cb, self._query_cb, None)
        # completions first, also those of a batch whose launch just failed
        buf = (V.VcCompletion * 64)()
        while True:
            got = V.lib.vc_sched_poll(C.c_void_p(self._h), buf, 64)
            for i in range(got):
                r = self._reqs.pop(buf[i].tag)
                r.done = buf[i].done
                r.hashed = bool(buf[i].hashed)
                r.status = int(buf[i].status)
                self.completed.append(r)
            if got < 64:
                break
        if self._error is not None:
            err, self._error = self._error, None
            raise err[1].with_traceback(err[2])
        V._check(min(n, 0), "vc_sched_pump")
        return n

    def idle(self) -> bool:
        return bool(V.lib.vc_sched_idle(C.c_void_p(self._h)))

    def _stats(self) -> V.VcSchedStats:
        st = V.VcSchedStats()
        V._check(V.lib.vc_sched_get_stats(C.c_void_p(self._h), C.byref(st)), "vc_sched_get_stats")
        return st

    @property
    def inflight_bytes(self) -> int:
        return int(self._stats().inflight_bytes)

    @property
    def inflight(self) -> List[None]:
        """One entry per batch in flight."""
        return [None] * int(self._stats().inflight_batches)

    @property
    def stream_inflight(self) -> Dict[str, int]:
        """The largest number of frames of one stream in flight."""
        return {"max": int(self._stats().max_stream_inflight)}


class Server:
    """The library's serving loop on the current GPU (vc_server): one sender
    and one receiver context per resolution class, ``max_inflight`` device
    streams per kind and class, the key state and scratch resident."""

    def __init__(self, key32: bytes, gamma: float, n: int, classes: Sequence[Tuple[int, int]], max_streams: int,
                 hbm_budget: int, max_inflight: int = 1, max_batch: int = 256, max_stream_inflight: int = 0,
                 hash_first: bool = False, parts: int = 1, side_streams: int = 0, scratch_slots: int = 2,
                 scratch_bytes: int = 0, max_inflight_hash: int = 0):
        self.key = V.vc_key_from_bytes(key32, gamma, n)
        self.classes = [(int(w), int(h)) for w, h in classes]
        cls = (C.c_uint32 * (2 * len(self.classes)))(*[v for wh in self.classes for v in wh])
        cfg = V.VcServerConfig(V.VcSchedConfig(int(hbm_budget), int(max_inflight), int(max_batch),
                                               int(max_stream_inflight), 1 if hash_first else 0,
                                               int(max_inflight_hash), 0),
                               int(max_streams), int(parts), int(side_streams), int(scratch_slots), int(scratch_bytes))
        h = C.c_void_p()
        V._check(V.lib.vc_server_create(C.byref(self.key), cls, len(self.classes), C.byref(cfg), C.byref(h)),
                 "vc_server_create")
        self._h = h.value

    def close(self) -> None:
        if self._h:
            V.lib.vc_server_destroy(C.c_void_p(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def request(tag: int, kind: str, stream: int, seq: int, frame, out, hashes, arrival: float = 0.0,
                nbytes: int = 0) -> V.VcRequest:
        """A vc_request for device tensors frame / out ((h, w, 3) uint8) and hashes (32 bytes)."""
        h, w = int(frame.shape[0]), int(frame.shape[1])
        return V.VcRequest(tag=tag, kind=0 if kind == "enc" else 1, stream=stream, seq=seq, w=w, h=h, cls=0,
                           nbytes=nbytes, arrival=arrival, frame=frame.data_ptr(), out=out.data_ptr(),
                           hash=hashes.data_ptr())

    def clock(self) -> float:
        return float(V.lib.vc_server_clock(C.c_void_p(self._h)))

    def submit(self, req: V.VcRequest) -> None:
        V._check(V.lib.vc_server_submit(C.c_void_p(self._h), C.byref(req)), "vc_server_submit")

    def pump(self) -> int:
        n = V.lib.vc_server_pump(C.c_void_p(self._h))
        V._check(min(n, 0), "vc_server_pump")
        return n

    def poll(self) -> List[V.VcCompletion]:
        out = []
        buf = (V.VcCompletion * 256)()
        while True:
            got = V.lib.vc_server_poll(C.c_void_p(self._h), buf, 256)
            out.extend(V.VcCompletion.from_buffer_copy(buf[i]) for i in range(got))
            if got < 256:
                return out

    def idle(self) -> bool:
        return bool(V.lib.vc_server_idle(C.c_void_p(self._h)))

    def stats(self) -> V.VcSchedStats:
        st = V.VcSchedStats()
        V._check(V.lib.vc_server_get_stats(C.c_void_p(self._h), C.byref(st)), "vc_server_get_stats")
        return st

    def run_trace(self, reqs: Sequence[V.VcRequest]):
        """Replays requests sorted by arrival (seconds from the call) in the
        library's own loop; returns the completions in the order of reqs."""
        arr = (V.VcRequest * max(len(reqs), 1))(*reqs)
        done = (V.VcCompletion * max(len(reqs), 1))()
        V._check(V.lib.vc_server_run_trace(C.c_void_p(self._h), len(reqs), arr, done), "vc_server_run_trace")
        return done

    def reset(self) -> None:
        """Every chain back to the key, every stream's next frame back to 0 (only when idle)."""
        V._check(V.lib.vc_server_reset(C.c_void_p(self._h)), "vc_server_reset")

    def status(self) -> int:
        return int(V.lib.vc_server_status(C.c_void_p(self._h)))
