"""Continuous-batching SRP server on one GPU.

Frames from many microphone arrays (different microphone counts and
candidate grids) arrive as requests. The server

* keeps every admitted array's geometry and tables resident on the device
  (srp_geometry) and admits an array only if its device footprint fits the
  memory budget; arrays that do not fit wait and are admitted when others
  close;
* runs a loop that, whenever one of its batch slots is free, takes every
  pending frame (up to 8 per array in FP32, 16 in BF16/FP16) into a batch: one
  host-to-device copy of the frames, per-array srp_gcc_samples_frames (FFT,
  PHAT phasors and GCC samples; the cross-spectra are formed on chip), then
  one ragged srp_map_nyquist_batched launch for all arrays of the batch;
* computes in FP32 (vector units) or BF16/FP16 (matrix cores, samples stored
  in that type, float32 accumulation), chosen per server;
* keeps two batch slots on two HIP streams, so a batch is assembled and its
  spectra run while the previous batch's maps are still on the GPU; requests
  that arrive meanwhile join the next batch (continuous batching); the slots'
  device and pinned host buffers are grown once after admissions to hold the
  largest batch, so no batch allocates memory while requests wait;
* validates each request (known, admitted array; frame shape; finite values)
  and fails that request alone on error; a failed batch launch fails only the
  requests of that batch;
* records per-frame latency from arrival to observed completion and, given a
  deadline, counts the frames that complete after it (and, if asked, fails
  frames whose deadline has already passed when a batch is assembled instead
  of computing them);
* takes an optional fault hook, called with each batch's requests before its
  device work is enqueued: an exception there fails that batch's requests
  alone, as a failed launch would (used to test the failure path).

In FP32, results do not depend on the batch a frame lands in: each GCC sample
and each candidate's map value is summed in a fixed order, whatever else is
batched. In BF16/FP16 a frame's map runs on the vector-unit or the
matrix-core kernel depending on how many frames of its array share the batch,
so its results agree with those of the same frame served alone to the
BF16/FP16 tolerance, not bit for bit.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import _lib as S


@dataclasses.dataclass
class Request:
    array_id: int
    seq: int
    frame: np.ndarray
    t_arrival: float
    status: str = "pending"          # pending | running | done | failed
    t_done: float = 0.0
    t_deadline: float = float("inf")
    missed: bool = False             # done after its deadline
    peak_index: int = -1
    peak_value: float = float("nan")
    error: str = ""

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class _Array:
    def __init__(self, array_id, geom: S.Geometry):
        self.id = array_id
        self.g = geom
        self.M, self.P, self.K, self.L, self.S, self.J = geom.M, geom.P, geom.K, geom.L, geom.S, geom.J
        self.pending: collections.deque = collections.deque()


def footprint(geom_J, M, K, L, S, P, h_max, max_f=S.BATCH_MAX_F, slots=2, sample_bytes=4):
    """Device bytes an array occupies in the server (geometry + its share of each slot):
    frames, per-microphone phasors (rows of K rounded up to 16 bins), samples and
    peaks per slot; candidates, the two GCC phase tables and the pair tables."""
    Kr = (K + 15) // 16 * 16
    slot = max_f * (M * L * 4 + M * Kr * 8 + S * sample_bytes + 16) + 4 * 256
    geom = 24 * geom_J + 2 * 8 * Kr * (2 * h_max + 34) + 64 * P + 4096
    return geom + slots * slot


class _Slot:
    def __init__(self, device):
        import torch
        self.device = device
        self.stream = torch.cuda.Stream(device=device)
        self.event = None
        self.requests: List[Request] = []
        self.cap = {}
        self.bufs = {}

    def buf(self, name, n, dtype):
        import torch
        if self.cap.get(name, 0) < n:
            # grow-only device buffers, kept for later batches
            self.bufs[name] = torch.empty(max(n, 2 * self.cap.get(name, 0)), dtype=dtype,
                                          device=self.device)
            self.cap[name] = self.bufs[name].numel()
        return self.bufs[name]

    def host(self, n):
        import torch
        if self.cap.get("host", 0) < n:
            self.bufs["host"] = torch.empty(max(n, 2 * self.cap.get("host", 0)),
                                            dtype=torch.float32, pin_memory=True)
            self.cap["host"] = self.bufs["host"].numel()
        return self.bufs["host"]


class SrpServer:
    def __init__(self, memory_budget: Optional[int] = None, device="cuda:0",
                 max_frames_per_array: Optional[int] = None, slots: int = 2,
                 dtype: str = "fp32", deadline_ms: Optional[float] = None,
                 shed_expired: bool = False,
                 fault_hook: Optional[Callable[[List[Request]], None]] = None):
        import torch
        if dtype not in ("fp32", "bf16", "fp16"):
            raise ValueError(f"dtype must be fp32, bf16 or fp16, not {dtype!r}")
        self.dtype = dtype
        self.sample_dtype = S.sample_torch_dtype(dtype)
        self.sample_bytes = 4 if dtype == "fp32" else 2
        self.device = torch.device(device)
        if memory_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            memory_budget = int(0.8 * free)
        self.budget = int(memory_budget)
        self.used = 0
        cap = S.batch_max_frames(dtype)
        self.max_f = cap if max_frames_per_array is None else min(int(max_frames_per_array), cap)
        self.arrays: Dict[int, _Array] = {}
        self.waiting: collections.OrderedDict = collections.OrderedDict()
        self.slots = [_Slot(self.device) for _ in range(slots)]
        self.completed: List[Request] = []
        self.failed: List[Request] = []
        self.rejected = 0
        self.deadline_s = None if deadline_ms is None else float(deadline_ms) * 1e-3
        self.shed_expired = bool(shed_expired)
        self.fault_hook = fault_hook
        self.deadline_misses = 0
        self.shed = 0
        self.failed_batches = 0
        self.batches = 0
        self.batch_frames: List[int] = []
        self._seq = 0
        self._reserved = True  # slot buffers cover max_f frames of every admitted array

    # ------------------------------------------------------------ admission
    def open_array(self, array_id, mic_xyz, candidates, *, fs, L, c=343.0, n_aux=2,
                   field="near", window="hann") -> bool:
        """Registers an array; returns True if admitted now, False if it waits for memory."""
        spec = dict(mic_xyz=mic_xyz, candidates=candidates, fs=fs, L=L, c=c, n_aux=n_aux,
                    field=field, window=window)
        N_p, off, Ssz = S.pair_layout(mic_xyz, c, fs / 2.0, n_aux)
        M = len(mic_xyz)
        K = L // 2 + 1
        need = footprint(len(candidates), M, K, L, Ssz, M * (M - 1) // 2,
                         int(N_p.max()) + n_aux, self.max_f, len(self.slots), self.sample_bytes)
        if need > self.budget:
            raise ValueError(f"array {array_id} needs {need} bytes, more than the whole budget")
        if self.used + need > self.budget:
            self.waiting[array_id] = (spec, need)
            return False
        self._admit(array_id, spec, need)
        return True

    def _admit(self, array_id, spec, need):
        g = S.Geometry(spec["mic_xyz"], spec["candidates"], fs=spec["fs"], L=spec["L"],
                       c=spec["c"], n_aux=spec["n_aux"], field=spec["field"],
                       window=spec["window"])
        a = _Array(array_id, g)
        a.need = need
        self.arrays[array_id] = a
        self.used += need
        self._reserved = False

    def close_array(self, array_id):
        a = self.arrays.pop(array_id, None)
        if a is not None:
            for r in a.pending:
                r.status, r.error = "failed", "array closed"
                self.failed.append(r)
            self.drain()
            a.g.close()
            self.used -= a.need
        self.waiting.pop(array_id, None)
        for wid in list(self.waiting):
            spec, need = self.waiting[wid]
            if self.used + need <= self.budget:
                del self.waiting[wid]
                self._admit(wid, spec, need)

    @property
    def admitted(self):
        return sorted(self.arrays)

    # ------------------------------------------------------------ requests
    def submit(self, array_id, frame, t_arrival: Optional[float] = None) -> Request:
        t = time.perf_counter() if t_arrival is None else t_arrival
        r = Request(array_id, self._seq, frame, t)
        if self.deadline_s is not None:
            r.t_deadline = t + self.deadline_s
        self._seq += 1
        a = self.arrays.get(array_id)
        err = ""
        if a is None:
            err = "array not admitted"
        elif not isinstance(frame, np.ndarray) or frame.shape != (a.M, a.L):
            err = f"frame must be a float32 array of shape ({a.M}, {a.L})"
        elif not np.all(np.isfinite(frame)):
            err = "frame has non-finite samples"
        if err:
            r.status, r.error, r.t_done = "failed", err, time.perf_counter()
            self.failed.append(r)
            self.rejected += 1
            return r
        r.frame = np.ascontiguousarray(frame, dtype=np.float32)
        a.pending.append(r)
        return r

    # ------------------------------------------------------------ the loop
    def pump(self) -> int:
        """Retires finished batches and launches a new one if a slot is free.

        Returns the number of requests completed by this call.
        """
        if not self._reserved:
            self._reserve()
        done = self._poll()
        if any(a.pending for a in self.arrays.values()):
            for slot in self.slots:
                if slot.event is None:
                    self._launch(slot)
                    break
        return done

    def drain(self):
        while any(s.event is not None for s in self.slots) or \
                any(a.pending for a in self.arrays.values()):
            self.pump()
            time.sleep(0)

    def _poll(self) -> int:
        n = 0
        for slot in self.slots:
            if slot.event is not None and slot.event.query():
                now = time.perf_counter()
                pk = slot.peaks_host
                for i, r in enumerate(slot.requests):
                    if r.status == "running":
                        r.status, r.t_done = "done", now
                        r.peak_index = int(pk[i, 0])
                        r.peak_value = float(pk[i:i + 1].view(np.int32)[0, 2].view(np.float32))
                        r.frame = None
                        if now > r.t_deadline:
                            r.missed = True
                            self.deadline_misses += 1
                        self.completed.append(r)
                        n += 1
                slot.event, slot.requests = None, []
        return n

    def _reserve(self):
        """Grows every slot's buffers to hold max_f frames of every admitted array
        (the share footprint() budgets), so that no batch allocates device or
        pinned host memory while requests wait (an allocation can stall the
        device for milliseconds)."""
        import torch
        fr = ws = xi = pk = 0
        for a in self.arrays.values():
            F = self.max_f
            fr += F * a.M * a.L
            ws += (a.g.workspace_bytes(F) + 255) // 256 * 256
            xi += F * a.S
            pk += F
        for slot in self.slots:
            slot.host(fr)
            slot.buf("frames", fr, torch.float32)
            slot.buf("ws", ws, torch.uint8)
            slot.buf("xi", xi, self.sample_dtype)
            slot.buf("peaks", 2 * pk, torch.int64)
            slot.buf("items", S.batched_workspace_bytes(len(self.arrays)), torch.uint8)
            if slot.cap.get("peaks_host", 0) < 2 * pk:
                slot.bufs["peaks_host"] = torch.empty(max(2 * pk, 256), dtype=torch.int64,
                                                      pin_memory=True)
                slot.cap["peaks_host"] = slot.bufs["peaks_host"].numel()
        self._reserved = True

    def _launch(self, slot: _Slot):
        import torch
        take = []
        now = time.perf_counter()
        for a in self.arrays.values():
            reqs = []
            while a.pending and len(reqs) < self.max_f:
                r = a.pending.popleft()
                if self.shed_expired and now > r.t_deadline:
                    # its deadline has passed: failed without computing it
                    r.status, r.error, r.t_done = "failed", "deadline passed", now
                    r.frame = None
                    self.failed.append(r)
                    self.shed += 1
                    continue
                reqs.append(r)
            if reqs:
                take.append((a, reqs))
        if not take:
            return
        # arena layout of this batch
        fr_off, ws_off, xi_off, pk_off = 0, 0, 0, 0
        plan = []
        for a, reqs in take:
            F = len(reqs)
            nws = a.g.workspace_bytes(F)
            plan.append((a, reqs, F, fr_off, ws_off, nws, xi_off, pk_off))
            fr_off += F * a.M * a.L
            ws_off += (nws + 255) // 256 * 256
            xi_off += F * a.S
            pk_off += F
        host = slot.host(fr_off)
        for a, reqs, F, fo, *_ in plan:
            hv = host[fo:fo + F * a.M * a.L].view(F, a.M, a.L).numpy()
            for j, r in enumerate(reqs):
                hv[j] = r.frame
                r.status = "running"
        frames = slot.buf("frames", fr_off, torch.float32)
        ws = slot.buf("ws", ws_off, torch.uint8)
        xi = slot.buf("xi", xi_off, self.sample_dtype)
        peaks = slot.buf("peaks", 2 * pk_off, torch.int64)
        item_ws = slot.buf("items", S.batched_workspace_bytes(len(plan)), torch.uint8)
        items = []
        reqs_all = []
        try:
            if self.fault_hook is not None:
                self.fault_hook([r for _, reqs, *_ in plan for r in reqs])
            with torch.cuda.stream(slot.stream):
                frames[:fr_off].copy_(host[:fr_off], non_blocking=True)
                for a, reqs, F, fo, wo, nws, xo, ko in plan:
                    fv = frames[fo:fo + F * a.M * a.L].view(F, a.M, a.L)
                    xv = xi[xo:xo + F * a.S].view(F, a.S)
                    S.gcc_samples_frames(a.g, fv, out=xv, dtype=self.dtype,
                                         workspace=ws[wo:wo + nws], stream=slot.stream)
                    items.append((a.g, xo, F, None, peaks[2 * ko:2 * (ko + F)].view(F, 2)))
                    reqs_all.extend(reqs)
                S.map_nyquist_batched(items, xi, item_ws, stream=slot.stream, dtype=self.dtype)
                if slot.cap.get("peaks_host", 0) < 2 * pk_off:
                    slot.bufs["peaks_host"] = torch.empty(max(2 * pk_off, 256), dtype=torch.int64,
                                                          pin_memory=True)
                    slot.cap["peaks_host"] = slot.bufs["peaks_host"].numel()
                ph = slot.bufs["peaks_host"][:2 * pk_off].view(pk_off, 2)
                ph.copy_(peaks[:2 * pk_off].view(pk_off, 2), non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(slot.stream)
        except Exception as e:  # a failed launch fails this batch only
            self.failed_batches += 1
            for _, reqs, *_ in plan:
                for r in reqs:
                    r.status, r.error, r.t_done = "failed", str(e), time.perf_counter()
                    r.frame = None
                    self.failed.append(r)
            return
        slot.peaks_host = ph.numpy()
        slot.requests = reqs_all
        slot.event = ev
        self.batches += 1
        self.batch_frames.append(len(reqs_all))

    # ------------------------------------------------------------ metrics
    def stats(self, t_span: float) -> dict:
        lat = np.asarray([r.latency for r in self.completed]) * 1e3
        evals = float(sum(self.arrays[r.array_id].J * self.arrays[r.array_id].P
                          for r in self.completed if r.array_id in self.arrays))
        return {
            "frames_done": len(self.completed), "frames_failed": len(self.failed),
            "rejected_requests": self.rejected, "failed_batches": self.failed_batches,
            "deadline_ms": None if self.deadline_s is None else self.deadline_s * 1e3,
            "deadline_misses": self.deadline_misses,
            "deadline_miss_rate": (self.deadline_misses / len(self.completed)
                                   if self.completed else 0.0),
            "shed_expired": self.shed,
            "frames_per_s": len(self.completed) / t_span,
            "cand_pair_evals_per_s": evals / t_span,
            "latency_ms_p50": float(np.percentile(lat, 50)) if lat.size else None,
            "latency_ms_p99": float(np.percentile(lat, 99)) if lat.size else None,
            "latency_ms_mean": float(lat.mean()) if lat.size else None,
            "batches": self.batches,
            "mean_frames_per_batch": float(np.mean(self.batch_frames)) if self.batch_frames else 0,
            "arrays_admitted": len(self.arrays), "arrays_waiting": len(self.waiting),
            "memory_budget_bytes": self.budget, "memory_used_bytes": self.used,
            "dtype": self.dtype, "max_frames_per_array": self.max_f,
        }
