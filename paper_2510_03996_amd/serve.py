"""Serving loop for encrypted CNN inference requests (continuous batching).

Requests of several resident models (e.g. a LeNet-5-shaped stack at N=2^14
and a ResNet-20-shaped chain at N=2^16, each with its evaluation keys and
preloaded weight plaintexts resident in HBM, the paper's preloading strategy
for keys and weights) arrive over time.  The scheduler

  * admits a waiting request when a slot (HIP stream + execution lane) is
    free and the byte footprint of the active requests plus the new one stays
    within the budget (resident keys and weights are accounted once);
  * advances every active request stage by stage (one layer per stage): a
    stage is enqueued asynchronously on the request's own stream as soon as
    the previous stage's completion event has fired, so requests that arrive
    while others are on the GPU overlap with them on the device;
  * records admission and completion times.

``sequential`` mode runs the same trace one request at a time (FIFO) on one
stream, the baseline the continuous mode is compared with.  Every stage runs
in the HIP library; this module only schedules.
"""
import collections
import time

import torch

from . import he


class Model:
    """A resident model: its library context and its stages.

    stages: list of callables ``stage(ct, stream) -> ct`` that enqueue one
    layer on ``stream`` and return the output ciphertext (device memory).
    footprint: device bytes one in-flight request of this model needs
    (its lane workspace, temporaries, input and output).
    key_ids: the model's evaluation keys (resident, or registered with host
    copies and loaded on demand by the library's key cache).
    """

    def __init__(self, name, ctx, stages, n_ct_buffers, footprint, key_ids=()):
        self.name, self.ctx, self.stages = name, ctx, stages
        self.n_ct_buffers = n_ct_buffers
        self.footprint = footprint
        self.key_ids = list(key_ids)


class Request:
    def __init__(self, rid, kind, arrival, ct):
        self.id, self.kind, self.arrival, self.input = rid, kind, float(arrival), ct
        self.cur = ct
        self.stage = 0
        self.event = None
        self.stream = None
        self.t_admit = self.t_done = None
        self.output = None
        # the input was written by work enqueued on the creating thread's
        # current stream (e.g. an asynchronous host-to-device fill); stage 0
        # runs on another stream and must wait for it
        self.ready = torch.cuda.Event()
        self.ready.record(torch.cuda.current_stream())

    @property
    def latency(self):
        return self.t_done - self.arrival


class Server:
    """layer_streams: streams (he_ctx_layer_streams) a stage may spread its
    convolution channels and hoisted key switches over while its request is
    the only one in flight (always in sequential mode); with several requests
    in flight each stage stays on its request's stream, since the requests
    already overlap and more streams than hardware queues make them wait on
    each other.  Results do not depend on it."""

    def __init__(self, models, slots=4, budget_bytes=None, layer_streams=2):
        self.models = models
        self.slots = slots
        self.budget = budget_bytes
        self.layer_streams = layer_streams
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        for s in self.streams:
            for m in models.values():
                m.ctx.lane_reserve(s, m.n_ct_buffers)
        self.max_active = 0
        self.max_bytes = 0

    def close(self):
        torch.cuda.synchronize()
        for s in self.streams:
            for m in self.models.values():
                m.ctx.lane_release(s)

    def _enqueue_stage(self, r, alone=True):
        m = self.models[r.kind]
        m.ctx.layer_streams(self.layer_streams if alone else 1)
        if r.stage == 0:
            r.stream.wait_event(r.ready)
        with torch.cuda.stream(r.stream):
            r.cur = m.stages[r.stage](r.cur, r.stream)
        r.stage += 1
        ev = torch.cuda.Event()
        ev.record(r.stream)
        r.event = ev

    def serve(self, requests, mode="continuous", t0=None):
        """Run requests (arrival times in seconds from t0); returns them completed."""
        try:
            return self._serve(requests, mode, t0)
        finally:
            for m in self.models.values():
                m.ctx.layer_streams(self.layer_streams)

    def _serve(self, requests, mode, t0):
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        done = []
        t0 = time.perf_counter() if t0 is None else t0
        if mode == "sequential":
            s = self.streams[0]
            while pending:
                r = pending.popleft()
                wait = r.arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                r.t_admit = time.perf_counter() - t0
                r.stream = s
                m = self.models[r.kind]
                while r.stage < len(m.stages):
                    self._enqueue_stage(r)
                r.event.synchronize()
                r.t_done = time.perf_counter() - t0
                r.output = r.cur
                done.append(r)
            return done
        free = list(self.streams)
        active = []
        used = 0
        while pending or active:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now and free:
                r = pending[0]
                fp = self.models[r.kind].footprint
                if self.budget is not None and active and used + fp > self.budget:
                    break
                pending.popleft()
                r.stream = free.pop()
                r.t_admit = now
                used += fp
                active.append(r)
            self.max_active = max(self.max_active, len(active))
            self.max_bytes = max(self.max_bytes, used)
            progressed = False
            for r in list(active):
                if r.event is not None and not r.event.query():
                    continue
                m = self.models[r.kind]
                if r.stage == len(m.stages):
                    r.t_done = time.perf_counter() - t0
                    r.output = r.cur
                    active.remove(r)
                    free.append(r.stream)
                    used -= m.footprint
                    done.append(r)
                else:
                    self._enqueue_stage(r, alone=len(active) == 1)
                progressed = True
            if not progressed:
                nxt = pending[0].arrival - (time.perf_counter() - t0) if pending else 0.0
                time.sleep(min(max(nxt, 0.0), 2e-4) if (pending and not active) else 5e-5)
        return done


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * p / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)
