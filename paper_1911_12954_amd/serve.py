"""Continuous-batching solve server for HOTRG and ATRG runs (beta/h scans
around T_c).

Requests (beta, h, Dcut, L, method) arrive over time.  The server

* admits a request while the device memory of the admitted runs stays
  within the HBM budget: each run's resident tensors (trg_resident_bytes)
  plus its join workspace (trg_workspace_bytes).  The runs of a lane share
  one workspace pool (trg_share_workspace); a HOTRG lane steps its
  same-shape runs in one batched call, which holds one workspace slot per
  run (each run brings its share), while an ATRG lane steps its runs one
  call after another through a single share; waiting requests are admitted
  as soon as finished runs free their memory;
* bounds the work of one lane round: a lane holds at most
  round_flops / (join flop of one step) runs (at least one), so a round of
  a large bond dimension stays short and the runs admitted first finish
  first instead of all sharing the device until the end of the stream;
  requests wait in arrival order, and one whose lane is full does not hold
  back requests of other lanes;
* keeps each run's tensors resident until it finishes;
* runs one lane (HIP stream) per (method, bond dimension), so lanes overlap
  on the device; inside a HOTRG lane, runs whose leg dims and next axis
  agree are stepped together by one batched library call
  (trg_hotrg_step_batch: one launch per kernel of the contraction and the
  normalisation for all of them, one eigensolver launch); ATRG runs take
  one call each (trg_atrg_step);
* advances a lane as soon as its previous step has completed (event query,
  no global barrier), and records arrival, admission and completion times.

Every result is computed by the same kernels in the same order as a run
alone, so it does not depend on what else is in the mix.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field


@dataclass
class Run:
    req: dict
    handle: object
    total: int
    done: int = 0
    t_admit: float = 0.0


@dataclass
class Lane:
    dcut: int
    stream: object
    runs: list = field(default_factory=list)
    event: object = None
    method: str = "hotrg"


class TrgBackend:
    """The HIP library through its Python binding."""

    def __init__(self, precision="fp32", d=4):
        import torch
        self.torch = torch
        self.precision = precision
        self.d = d

    def _precision(self, method):
        """ATRG contracts in FP64 or FP32: a server with a split-BF16 join
        (BF16x3 or BF16x6) runs its ATRG requests with FP32 contractions."""
        return "fp32" if method == "atrg" and self.precision in ("bf16x3", "bf16x6") else self.precision

    def resident(self, req) -> int:
        from .trg import trg_resident_bytes
        method = req.get("method", "hotrg")
        return trg_resident_bytes(self.d, req["dcut"], self._precision(method), method)

    def workspace(self, dcut, method="hotrg") -> int:
        from .trg import trg_workspace_bytes
        return trg_workspace_bytes(self.d, dcut, self._precision(method), method)

    def step_flops(self, dcut, method="hotrg") -> float:
        """Flop of one steady-state step: the HOTRG join 2 Dcut^(4d-1); for
        ATRG the contraction 4 Dcut^(2d+1) plus the randomized SVD's
        (4 Dcut + 2) products of 2 Dcut^(d+2) x 5 Dcut flop."""
        D = float(dcut)
        if method == "atrg":
            return 4.0 * D ** (2 * self.d + 1) + (4.0 * D + 2.0) * 2.0 * D ** (self.d + 2) * 5.0 * D
        return 2.0 * D ** (4 * self.d - 1)

    def new_lane(self, dcut):
        return self.torch.cuda.Stream()

    def create(self, req, stream, donor=None):
        """A run on the lane's stream; its join plan is sized to the lane's
        workspace, which it shares with `donor` (a live run of the lane)."""
        from .trg import trg_init_ising, trg_share_workspace
        method = req.get("method", "hotrg")
        h = trg_init_ising(req["beta"], req["h"], self.d, dcut=req["dcut"], precision=self._precision(method),
                           method=method, stream=stream, workspace_bytes=self.workspace(req["dcut"], method))
        if donor is not None:
            trg_share_workspace(h, donor)
        return h

    def dims(self, h):
        return h.dims()[0]

    def step(self, handles, axis, dcut, method="hotrg"):
        from .trg import trg_hotrg_step_batch
        if method == "atrg":
            for h in handles:
                h.atrg_step(axis, dcut)
        elif len(handles) == 1:
            handles[0].hotrg_step(axis, dcut)
        else:
            trg_hotrg_step_batch(handles, axis, dcut)

    def mark(self, stream):
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return ev

    def ready(self, ev) -> bool:
        return ev is None or ev.query()

    def result(self, h) -> float:
        return h.free_energy()

    def close(self, h):
        h.close()


class Server:
    def __init__(self, backend, hbm_budget: int, d: int = 4, max_batch: int = 64,
                 round_flops: float = 4e13, max_active: int = 256):
        self.be = backend
        self.budget = int(hbm_budget)
        self.d = d
        self.max_batch = max_batch
        self.round_flops = float(round_flops)
        self.max_active = int(max_active)
        self.lanes = {}
        self.used = 0
        self.peak_used = 0
        self.results = []
        self.batch_calls = 0
        self.batched_runs = 0

    def _lane(self, method, dcut):
        key = (method, dcut)
        if key not in self.lanes:
            self.lanes[key] = Lane(dcut, self.be.new_lane(dcut), method=method)
        return self.lanes[key]

    def lane_cap(self, dcut, method="hotrg") -> int:
        """Runs a lane holds at once."""
        return max(1, min(self.max_active, int(self.round_flops // self.be.step_flops(dcut, method=method))))

    def _admit(self, req, now):
        """Admit `req` if its lane has room and the memory fits.  Returns
        True (admitted), "lane" (its lane is full) or False (no memory)."""
        method = req.get("method", "hotrg")
        res = self.be.resident(req)
        ws = self.be.workspace(req["dcut"], method=method)
        if res + ws > self.budget:
            raise ValueError(f"request {req['id']} needs {res + ws} bytes, more than the whole budget")
        lane = self.lanes.get((method, req["dcut"]))
        if lane is not None and len(lane.runs) >= self.lane_cap(req["dcut"], method):
            return "lane"
        need = res + self._share(method, ws, lane)
        if self.used + need > self.budget:
            return False
        lane = self._lane(method, req["dcut"])
        donor = lane.runs[0].handle if lane.runs else None
        h = self.be.create(req, lane.stream, donor)
        m = req["L"].bit_length() - 1
        lane.runs.append(Run(req, h, self.d * m, 0, now))
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        return True

    @staticmethod
    def _share(method, ws, lane):
        """Workspace bytes a new run adds to its lane: a HOTRG run its own
        slot of the batched step, an ATRG run nothing once its lane has one."""
        if method == "atrg" and lane is not None and lane.runs:
            return 0
        return ws

    def _release(self, lane, req):
        """Bytes a finished run of `lane` frees (its share and residents)."""
        freed = self.be.resident(req)
        if lane.method != "atrg":
            freed += self.be.workspace(lane.dcut, method=lane.method)
        return freed

    def _advance(self, lane, now, t0):
        """Finish completed runs of a lane whose last step is done, then issue
        the next step of every remaining run (batched by leg dims)."""
        if not self.be.ready(lane.event):
            return False
        lane.event = None
        had_runs = bool(lane.runs)
        still = []
        for run in lane.runs:
            if run.done >= run.total:
                lnz = self.be.result(run.handle)
                self.be.close(run.handle)
                self.used -= self._release(lane, run.req)
                t_done = time.perf_counter() - t0
                self.results.append({"id": run.req["id"], "lnz": lnz, "arrival": run.req["arrival"],
                                     "admitted": run.t_admit, "done": t_done,
                                     "latency": t_done - run.req["arrival"], "dcut": run.req["dcut"],
                                     "method": lane.method,
                                     "L": run.req["L"], "beta": run.req["beta"], "h": run.req["h"]})
            else:
                still.append(run)
        if had_runs and not still and lane.method == "atrg":
            self.used -= self.be.workspace(lane.dcut, method=lane.method)   # the last user freed it
        lane.runs = still
        if not still:
            return True
        groups = {}
        for run in still:
            axis = run.done % self.d
            key = (tuple(self.be.dims(run.handle)), axis)
            groups.setdefault(key, []).append(run)
        for (dims, axis), runs in groups.items():
            for i in range(0, len(runs), self.max_batch):
                chunk = runs[i:i + self.max_batch]
                self.be.step([r.handle for r in chunk], axis, lane.dcut, method=lane.method)
                self.batch_calls += 1
                self.batched_runs += len(chunk)
                for r in chunk:
                    r.done += 1
        lane.event = self.be.mark(lane.stream)
        return True

    def serve(self, requests, window: float = None, idle_sleep: float = 5e-4):
        """Process `requests` (dicts with an 'arrival' time in seconds) in
        real time until all are done or `window` seconds have passed.
        Returns a summary with completed solves/s and latency percentiles."""
        pending = sorted(requests, key=lambda r: r["arrival"])
        waiting = []
        t0 = time.perf_counter()
        i = 0
        while True:
            now = time.perf_counter() - t0
            if window is not None and now >= window:
                break
            while i < len(pending) and pending[i]["arrival"] <= now:
                waiting.append(pending[i])
                i += 1
            # first come, first served while memory allows; a request whose
            # lane is full is passed over
            keep = []
            for j, req in enumerate(waiting):
                got = self._admit(req, now)
                if got is False:
                    keep += waiting[j:]
                    break
                if got == "lane":
                    keep.append(req)
            waiting = keep
            progressed = False
            for lane in list(self.lanes.values()):
                progressed |= self._advance(lane, now, t0)
            active = sum(len(l.runs) for l in self.lanes.values())
            if i >= len(pending) and not waiting and active == 0:
                break
            if not progressed:
                time.sleep(idle_sleep)
        elapsed = time.perf_counter() - t0
        return self.summary(elapsed, len(requests))

    def summary(self, elapsed, submitted):
        import numpy as np
        lat = np.array([r["latency"] for r in self.results]) if self.results else np.zeros(0)
        active = sum(len(l.runs) for l in self.lanes.values())
        return {
            "submitted": submitted,
            "completed": len(self.results),
            "censored_active": active,
            "elapsed_s": elapsed,
            "solves_per_s": len(self.results) / elapsed if elapsed > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "peak_footprint_bytes": self.peak_used,
            "budget_bytes": self.budget,
            "step_calls": self.batch_calls,
            "mean_runs_per_call": self.batched_runs / self.batch_calls if self.batch_calls else 0.0,
        }

    def close(self):
        for lane in self.lanes.values():
            for run in lane.runs:
                self.be.close(run.handle)
                self.used -= self._release(lane, run.req)
            if lane.runs and lane.method == "atrg":
                self.used -= self.be.workspace(lane.dcut, method=lane.method)
            lane.runs = []
