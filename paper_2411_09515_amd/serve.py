"""Continuous-batching service of frames from several detectors.

Frames arrive from each detector into a device-resident ingest ring (as a
detector writing straight into GPU memory would deliver them) and are served
to completion: corrected, clipped, sparsified and peak-picked (the whole
path), with the kept pixels, the peaks and the profile returned to the host.

Scheduling:
* every detector owns a set of *slots*, each the device memory of one
  in-flight batch (frames, profile, workspace, outputs), and one stream
  (default priority); the number of slots comes from an HBM budget
  (admission by memory);
* whenever a slot is free and its detector has frames waiting, the waiting
  frames (up to the slot's batch size) are admitted as one batch and
  launched at once, while other batches are still running: batches of
  different detectors, and successive batches of one detector, overlap on
  the device;
* a batch completes in two steps: the per-frame counts come back, then
  exactly the kept pixels and peaks; the slot is then free again.

Per-frame latency is measured from the frame's arrival to the moment its
results are on the host.  Every step of the path runs in the library's HIP
kernels; this module only schedules them.
"""

from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api
from . import binding as B


@dataclass
class Request:
    """One frame: detector, index of its raw frame in the detector's ingest
    ring, arrival time (s, on the server's clock)."""

    det: int
    ring_index: int
    t_arrival: float
    rid: int = 0
    t_done: float = float("nan")
    batch_size: int = 0
    n_kept: int = 0
    kept_index: np.ndarray = field(default=None, repr=False)
    kept_value: np.ndarray = field(default=None, repr=False)
    n_peaks: int = 0
    peaks: np.ndarray = field(default=None, repr=False)
    mean: np.ndarray = field(default=None, repr=False)
    std: np.ndarray = field(default=None, repr=False)
    # the rest of the profile, returned only by a Server with full_profile=True
    sem: np.ndarray = field(default=None, repr=False)
    sum_w: np.ndarray = field(default=None, repr=False)
    n_members: np.ndarray = field(default=None, repr=False)
    n_iter: np.ndarray = field(default=None, repr=False)
    converged: np.ndarray = field(default=None, repr=False)


class Detector:
    """A detector's resident state: geometry, calibration, ingest ring."""

    def __init__(self, name, geom: api.Geometry, pedestal, gain, ring_raw, params: api.Params, max_batch=8,
                 kept_capacity=None, peak_capacity=4096):
        self.name, self.geom, self.params = name, geom, params
        self.pedestal, self.gain = pedestal, gain
        self.ring = ring_raw            # device [K, N] raw words (int16 view of uint16)
        self.max_batch = int(max_batch)
        # kept pixels per frame: 1/16 of the detector by default (about 1.8 % are kept at 3 sigma)
        self.kept_capacity = int(geom.n_pix // 16 if kept_capacity is None else kept_capacity)
        self.peak_capacity = int(peak_capacity)

    def slot_bytes(self):
        N, nb, B_ = self.geom.n_pix, self.geom.n_bins, self.max_batch
        ws = api.workspace_bytes(B_, N, nb)
        # frames, profile, results and their packed copies, counts
        per = (self.geom.frame_words * 4 + nb * (4 * 8 + 3 * 4) + 2 * (self.kept_capacity * 8 + self.peak_capacity * B.PEAK_BYTES)
               + 32)
        return B_ * per + ws


class _Slot:
    def __init__(self, det: Detector, device, stream, full_profile=False, n_arenas=1):
        F, nb = det.max_batch, det.geom.n_bins
        self.det = det
        self.full_profile = full_profile
        self.frames = torch.empty((F, det.geom.frame_words), dtype=torch.float32, device=device)
        self.n_invalid = torch.empty(F, dtype=torch.int64, device=device)
        self.profile = api.new_profile(F, nb, device)
        self.workspace = api.new_workspace(F, det.geom, device)
        self.out = dict(kept_index=torch.empty((F, det.kept_capacity), dtype=torch.int32, device=device),
                        kept_value=torch.empty((F, det.kept_capacity), dtype=torch.float32, device=device),
                        n_kept=torch.empty(F, dtype=torch.int64, device=device),
                        peaks=torch.empty((F, det.peak_capacity, B.PEAK_BYTES), dtype=torch.uint8,
                                          device=device),
                        n_peaks=torch.empty(F, dtype=torch.int64, device=device))
        # every frame's results packed back to back (one copy per kind to the host)
        self.packed = dict(offsets=torch.empty(2 * (F + 1), dtype=torch.int64, device=device),
                           index=torch.empty(F * det.kept_capacity, dtype=torch.int32, device=device),
                           value=torch.empty(F * det.kept_capacity, dtype=torch.float32, device=device),
                           peaks=torch.empty((F * det.peak_capacity, B.PEAK_BYTES), dtype=torch.uint8,
                                             device=device))
        self.h_idx = torch.empty(F, dtype=torch.int64, pin_memory=True)
        self.d_idx = torch.empty(F, dtype=torch.int64, device=device)
        self.h_counts = torch.empty((2, F), dtype=torch.int64, pin_memory=True)
        self.h_offsets = torch.empty(2 * (F + 1), dtype=torch.int64, pin_memory=True)
        # results land in one of n_arenas pinned host arenas, in turn per batch
        rest = ("sem", "sum_w", "n_members", "n_iter", "converged") if full_profile else ()
        self.arenas = []
        for _ in range(n_arenas):
            a = dict(mean=torch.empty((F, nb), dtype=torch.float64, pin_memory=True),
                     std=torch.empty((F, nb), dtype=torch.float64, pin_memory=True),
                     index=torch.empty(F * det.kept_capacity, dtype=torch.int32, pin_memory=True),
                     value=torch.empty(F * det.kept_capacity, dtype=torch.float32, pin_memory=True),
                     peaks=torch.empty((F * det.peak_capacity, B.PEAK_BYTES), dtype=torch.uint8, pin_memory=True))
            for k in rest:
                a[k] = torch.empty((F, nb), dtype=self.profile[k].dtype, pin_memory=True)
            self.arenas.append(a)
        self.rest = rest
        self.arena = 0
        # touch every page of the pinned buffers now: first touches fault, and
        # would otherwise land inside the serving loop
        for t in (self.h_idx, self.h_counts, self.h_offsets, *(t for a in self.arenas for t in a.values())):
            t.zero_()
        self.stream = stream
        self.graphs = {}     # batch size -> captured device work of one batch
        self.ev_counts = torch.cuda.Event()
        self.ev_done = torch.cuda.Event()
        self.batch = []
        self.phase = 0   # 0 free, 1 computing, 2 copying results

    def device_work(self, F):
        """The whole path on the first F ring frames named by d_idx, on the
        current stream: correct (reading the ring frames where they lie),
        clip, classify, pack."""
        d = self.det
        frames = self.frames[:F]
        api.correct_indexed(d.ring, self.d_idx[:F], d.pedestal, d.gain, d.geom.norm, out=frames,
                            n_invalid=self.n_invalid[:F], geom=d.geom)
        prof = {k: v[:F] for k, v in self.profile.items()}
        api.sigma_clip(frames, d.geom, d.params, out=prof)
        out = {k: v[:F] for k, v in self.out.items()}
        api.classify(frames, d.geom, prof, d.params, d.kept_capacity, d.peak_capacity,
                     workspace=self.workspace, out=out)
        packed = dict(offsets=self.packed["offsets"][:2 * (F + 1)], index=self.packed["index"],
                      value=self.packed["value"], peaks=self.packed["peaks"])
        api.pack_results(out, d.kept_capacity, d.peak_capacity, packed)


def _keep_result_buffers_on_the_heap():
    """Results handed to the host are fresh arrays of a few hundred KB per
    frame; glibc serves such sizes with a new mapping each time (every page
    faults on first touch) until its adaptive threshold has grown, and hands
    freed heap back to the system.  Fixing both thresholds keeps results on
    heap pages that, once touched, stay mapped: a serving process reaches a
    steady state without page faults on the result path."""
    try:
        libc = ctypes.CDLL("libc.so.6")
    except OSError:
        return False
    M_TRIM_THRESHOLD, M_MMAP_THRESHOLD = -1, -3
    ok = libc.mallopt(M_MMAP_THRESHOLD, 32 << 20) == 1
    ok = libc.mallopt(M_TRIM_THRESHOLD, -1) == 1 and ok   # never hand freed heap back
    return ok


class Server:
    """Continuous batching over detectors within an HBM budget (bytes).

    With ``copy_results`` (default) every request's result arrays are its
    own copies.  Without it they are views into the slot's pinned result
    arenas (two per slot, used in turn), valid until that slot has finished
    its next batch: a consumer that stores or forwards each result as it
    completes avoids one host copy of every kept pixel.  With
    ``tune_malloc`` (default) the process's malloc thresholds are set so
    that per-request result copies come from the heap (see
    ``_keep_result_buffers_on_the_heap``)."""

    def __init__(self, detectors, hbm_budget=8 << 30, device="cuda", max_slots_per_detector=2, tune_malloc=True,
                 full_profile=False, copy_results=True):
        self.copy_results = copy_results
        if tune_malloc:
            _keep_result_buffers_on_the_heap()
        self.detectors = list(detectors)
        self.device = torch.device(device)
        self.slots = []
        # admission by memory: slots for each detector while the budget lasts,
        # round robin so that every detector gets at least one.  Two per
        # detector by default: one batch running and one queued behind it on
        # the detector's stream; more slots only queue more single-frame
        # batches, while with two the frames that arrive meanwhile wait on
        # the host and leave together in the next, larger batch.
        used = 0
        per_det = [0] * len(self.detectors)
        # one stream per detector: a detector's batches queue in order, different
        # detectors' batches run side by side (the device has few hardware queues,
        # so more streams than detectors would only make batches wait behind others)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in self.detectors]
        progress = True
        while progress:
            progress = False
            for i, d in enumerate(self.detectors):
                b = d.slot_bytes()
                if per_det[i] < max_slots_per_detector and used + b <= hbm_budget:
                    self.slots.append(_Slot(d, self.device, self.streams[i], full_profile,
                                            1 if copy_results else 2))
                    per_det[i] += 1
                    used += b
                    progress = True
        if any(n == 0 for n in per_det):
            raise MemoryError("the HBM budget does not hold one batch of every detector")
        self.slots_per_detector = per_det
        self.reserved_bytes = used

    # -- one batch -----------------------------------------------------------------------

    def _launch(self, slot: _Slot, batch):
        F = len(batch)
        for f, r in enumerate(batch):
            slot.h_idx[f] = r.ring_index
        with torch.cuda.stream(slot.stream):
            slot.d_idx[:F].copy_(slot.h_idx[:F], non_blocking=True)
            g = slot.graphs.get(F)
            if g is not None:
                g.replay()
            else:
                slot.device_work(F)
            slot.h_offsets[:2 * (F + 1)].copy_(slot.packed["offsets"][:2 * (F + 1)], non_blocking=True)
            slot.h_counts[0, :F].copy_(slot.out["n_kept"][:F], non_blocking=True)
            slot.h_counts[1, :F].copy_(slot.out["n_peaks"][:F], non_blocking=True)
            A = slot.arenas[slot.arena]
            for k in ("mean", "std", *slot.rest):
                A[k][:F].copy_(slot.profile[k][:F], non_blocking=True)
            slot.ev_counts.record(slot.stream)
        slot.batch = batch
        slot.phase = 1

    def _fetch(self, slot: _Slot):
        F = len(slot.batch)
        tk = int(slot.h_offsets[F])
        tp = int(slot.h_offsets[2 * F + 1])
        with torch.cuda.stream(slot.stream):
            # exactly the packed results: one contiguous copy per kind
            A = slot.arenas[slot.arena]
            if tk:
                A["index"][:tk].copy_(slot.packed["index"][:tk], non_blocking=True)
                A["value"][:tk].copy_(slot.packed["value"][:tk], non_blocking=True)
            if tp:
                A["peaks"][:tp].copy_(slot.packed["peaks"][:tp], non_blocking=True)
            slot.ev_done.record(slot.stream)
        slot.phase = 2

    def _finish(self, slot: _Slot, now):
        F = len(slot.batch)
        A = slot.arenas[slot.arena]
        counts = slot.h_counts[:, :F].numpy()
        off = slot.h_offsets[:2 * (F + 1)].numpy()
        for f, r in enumerate(slot.batch):
            k0, k1 = int(off[f]), int(off[f + 1])
            p0, p1 = int(off[F + 1 + f]), int(off[F + 2 + f])
            r.n_kept, r.n_peaks = int(counts[0, f]), int(counts[1, f])
            r.kept_index = A["index"][k0:k1].numpy().view(np.uint32)
            r.kept_value = A["value"][k0:k1].numpy()
            r.peaks = A["peaks"][p0:p1].numpy().reshape(-1).view(api.PEAK_DTYPE)
            r.mean = A["mean"][f].numpy()
            r.std = A["std"][f].numpy()
            for k in slot.rest:
                setattr(r, k, A[k][f].numpy())
            if self.copy_results:
                for k in ("kept_index", "kept_value", "peaks", "mean", "std", *slot.rest):
                    setattr(r, k, getattr(r, k).copy())
            r.batch_size = F
            r.t_done = now
        slot.batch = []
        slot.phase = 0
        slot.arena = (slot.arena + 1) % len(slot.arenas)

    def capture_graphs(self):
        """Capture every slot's device work for every batch size as a HIP
        graph (one launch per batch instead of one per kernel).  The graphs
        hold no copies to the host and no memory sets."""
        torch.cuda.synchronize(self.device)
        # the server owns its graphs until close(); no graph is destroyed while
        # a capture is open (api.capturing defers releases, pauses collection)
        with api.capturing():
            for s in self.slots:
                api.release_graphs(s.graphs)
                for F in range(1, s.det.max_batch + 1):
                    s.d_idx[:F].zero_()
                    with torch.cuda.stream(s.stream):
                        s.device_work(F)          # eager run first: nothing is initialised inside the capture
                    s.stream.synchronize()
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=s.stream):
                        s.device_work(F)
                    s.graphs[F] = g
        torch.cuda.synchronize(self.device)

    def close(self):
        """Release the captured graphs (before the device buffers they use;
        deferred while a capture is open)."""
        torch.cuda.synchronize(self.device)
        for s in self.slots:
            api.release_graphs(s.graphs)

    def warmup(self, graphs=True):
        """Graphs for every slot and batch size (unless ``graphs`` is False),
        then one batch of one frame and one full batch per detector, so that
        the first served frames pay for neither capture nor kernel loading."""
        if graphs:
            self.capture_graphs()
        reqs = []
        for d_i, d in enumerate(self.detectors):
            reqs.append(Request(det=d_i, ring_index=0, t_arrival=0.0))
        self.run(reqs, realtime=False)
        reqs = [Request(det=d_i, ring_index=k % d.ring.shape[0], t_arrival=0.0)
                for d_i, d in enumerate(self.detectors) for k in range(d.max_batch)]
        self.run(reqs, realtime=False)

    # -- the loop ------------------------------------------------------------------------

    def run(self, requests, realtime=True, idle_sleep=20e-6):
        """Serve ``requests`` (sorted by arrival); with ``realtime`` a request is
        visible only from its arrival time on.  Returns the requests, completed,
        and a dict of run statistics."""
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        for i, r in enumerate(reqs):
            r.rid = i
        waiting = [collections.deque() for _ in self.detectors]
        det_index = {id(d): i for i, d in enumerate(self.detectors)}
        nxt, done = 0, 0
        max_wait, n_batches, max_busy = 0, 0, 0
        t0 = time.perf_counter()
        while done < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(reqs) and (not realtime or reqs[nxt].t_arrival <= now):
                waiting[reqs[nxt].det].append(reqs[nxt])
                nxt += 1
            busy = False
            for s in self.slots:
                if s.phase == 1 and s.ev_counts.query():
                    self._fetch(s)
                    busy = True
                if s.phase == 2 and s.ev_done.query():
                    done += len(s.batch)
                    self._finish(s, time.perf_counter() - t0)
                    busy = True
            for s in self.slots:
                if s.phase != 0:
                    continue
                q = waiting[det_index[id(s.det)]]
                if not q:
                    continue
                batch = [q.popleft() for _ in range(min(len(q), s.det.max_batch))]
                self._launch(s, batch)
                n_batches += 1
                busy = True
            max_wait = max(max_wait, sum(len(q) for q in waiting))
            max_busy = max(max_busy, sum(1 for s in self.slots if s.phase != 0))
            if not busy and idle_sleep:
                time.sleep(idle_sleep)
        wall = time.perf_counter() - t0
        lat = np.array([r.t_done - r.t_arrival for r in reqs]) * 1e3
        stats = dict(frames=len(reqs), wall_s=wall, batches=n_batches, max_waiting=max_wait,
                     max_batches_in_flight=max_busy,
                     mean_batch=len(reqs) / max(1, n_batches),
                     latency_ms={"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                                 "max": float(lat.max())} if len(lat) else None,
                     slots_per_detector=self.slots_per_detector, reserved_bytes=self.reserved_bytes)
        return reqs, stats


def poisson_arrivals(rates_hz, duration_s, ring_sizes, seed=0):
    """Requests with Poisson arrivals per detector (rates in Hz) over
    ``duration_s``; each request points at the next frame of its ring."""
    rng = np.random.default_rng(seed)
    out = []
    for d, (rate, k) in enumerate(zip(rates_hz, ring_sizes)):
        t, n = 0.0, 0
        while True:
            t += rng.exponential(1.0 / rate)
            if t >= duration_s:
                break
            out.append(Request(det=d, ring_index=n % k, t_arrival=t))
            n += 1
    return sorted(out, key=lambda r: r.t_arrival)
