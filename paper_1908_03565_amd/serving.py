"""Continuous-batching decode server over the batch entry points.

Requests (one frame each: coefficient planes, maps and parameters in host
memory) arrive over time.  The server

  * admits waiting requests in arrival order while their device footprint
    (inputs, workspace, outputs) fits the HBM budget;
  * uploads each admitted request's inputs (pinned host memory) on an upload
    stream, asynchronously;
  * gathers every uploaded request that is not yet running into one batch
    and launches it (block info, reconstruction, EPF passes, finish as
    persistent kernels over the batch's tiles) on the next of several compute
    streams, so batches that start while others still run overlap on the
    device;
  * copies each finished request's output back to host memory and frees its
    budget.

A request's latency runs from its arrival time to the completion of that
copy.  All device work goes through the C-ABI library; this module only
schedules, allocates (torch) and moves data.
"""
import collections
import threading
import time

import numpy as np

from . import jxlr as J

_OUT_BYTES = {0: 4, 1: 1, 2: 2}


_ALLOC = 512  # torch's caching allocator rounds every block up to this


def _rounded(n):
    return -(-n // _ALLOC) * _ALLOC


# the optional inputs a request may carry (patches, dots, DcQuantField,
# splines), each uploaded as one tensor of its own
_OPTIONAL = ("patch_place", "patch_samples", "dots", "dc_quant", "spline_offsets",
             "spline_points", "spline_dct")


def footprint_bytes(p, frame=None):
    """Device bytes one request holds while admitted, each buffer rounded as
    the allocator rounds it: the AC (int32) and DC planes, the three maps,
    the chroma-from-luma tiles, the optional inputs of `frame` (if given),
    the output planes, and its part of the batch workspace (the library's
    per-frame workspace plus its share of the descriptor header: a frame
    descriptor, one int per 64x32 tile, its prefix entries and its option
    stage entries, which is what a batch of this frame alone adds over
    jxlr_workspace_bytes)."""
    W, H = p.xsize, p.ysize
    Wb, Hb = (W + 7) // 8, (H + 7) // 8
    Wt, Ht = (W + 63) // 64, (H + 63) // 64
    inputs = (_rounded(3 * 64 * Wb * Hb * 4) + _rounded(3 * Wb * Hb * 4) + 3 * _rounded(Wb * Hb) +
              2 * _rounded(Wt * Ht * 4))
    if frame is not None:
        for k in _OPTIONAL:
            a = frame.get(k)
            if a is not None and len(a):
                nb = a.numel() * a.element_size() if hasattr(a, "numel") else np.asarray(a).size * 4
                inputs += _rounded(nb)
    out = _rounded(3 * W * H * _OUT_BYTES[p.out_format])
    return inputs + out + J.batch_workspace_bytes([p])


class Request:
    __slots__ = ("rid", "t_arrival", "frame", "params", "fp", "df", "out", "host_out", "ev_up",
                 "ev_done", "t_done", "keep")

    def __init__(self, rid, t_arrival, frame, params, keep=False):
        self.rid = rid
        self.t_arrival = t_arrival
        self.frame = frame
        self.params = params
        self.fp = footprint_bytes(params, frame)
        self.df = self.out = self.host_out = self.ev_up = self.ev_done = None
        self.t_done = None
        self.keep = keep


class Server:
    """One device, one context.  budget_bytes bounds the summed footprint of
    admitted requests; max_batch bounds the requests per launched batch;
    n_streams compute streams take batches in turn."""

    def __init__(self, ctx, budget_bytes, max_batch=64, n_streams=2):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.dev = f"cuda:{ctx.device}"
        self.budget = budget_bytes
        self.max_batch = max_batch
        # default-priority streams only
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(n_streams)]
        self.up_stream = torch.cuda.Stream(device=self.dev)
        self.down_stream = torch.cuda.Stream(device=self.dev)
        # batch descriptors are written on a stream of their own, which the
        # prepare call synchronizes (only its own copies are ever on it)
        self.prep_stream = torch.cuda.Stream(device=self.dev)
        self.next_stream = 0
        self.used = 0
        self.peak_used = 0
        self.waiting = collections.deque()   # arrived, not admitted
        self.uploaded = []                   # admitted and uploaded, not launched
        self.running = []                    # (event, requests, keepalive)
        self.copying = []                    # requests whose output copy is queued
        self.done = []
        self.batches = 0
        self.batch_sizes = []

    # -- stages -------------------------------------------------------------
    def _admit(self):
        torch = self.torch
        while self.waiting and self.used + self.waiting[0].fp <= self.budget:
            r = self.waiting.popleft()
            self.used += r.fp
            self.peak_used = max(self.peak_used, self.used)
            with torch.cuda.stream(self.up_stream):
                # pinned planes upload asynchronously; the request keeps them
                # until its output is back
                r.df = J.DeviceFrame(r.frame, device=self.dev, non_blocking=True)
                r.out = self.ctx.empty_out(r.params)
                r.ev_up = torch.cuda.Event()
                r.ev_up.record(self.up_stream)
            self.uploaded.append(r)
        if self.waiting and not self.uploaded and not self.running and not self.copying:
            # nothing in flight and the head does not fit: it can never fit
            r = self.waiting[0]
            raise RuntimeError(f"request {r.rid} needs {r.fp} bytes, over the budget {self.budget}")

    def _launch(self):
        torch = self.torch
        while self.uploaded:
            batch, self.uploaded = self.uploaded[:self.max_batch], self.uploaded[self.max_batch:]
            s = self.streams[self.next_stream]
            self.next_stream = (self.next_stream + 1) % len(self.streams)
            ps = [r.params for r in batch]
            with torch.cuda.stream(s):
                for r in batch:
                    s.wait_event(r.ev_up)
                # a fresh workspace per batch, held until the batch is done
                ws = self.ctx.batch_workspace(ps)
                plan = self.ctx.batch_prepare(ps, [r.df.io(r.out) for r in batch], ws,
                                              stream=self.prep_stream)
                self.ctx.batch_run(plan, stream=s)
                ev = torch.cuda.Event()
                ev.record(s)
            self.running.append((ev, batch, (ws, plan)))
            self.batches += 1
            self.batch_sizes.append(len(batch))

    def _complete(self, now_fn):
        torch = self.torch
        still = []
        for ev, batch, keep in self.running:
            if not ev.query():
                still.append((ev, batch, keep))
                continue
            with torch.cuda.stream(self.down_stream):
                self.down_stream.wait_event(ev)
                for r in batch:
                    r.host_out = torch.empty(r.out.shape, dtype=r.out.dtype, pin_memory=True)
                    r.host_out.copy_(r.out, non_blocking=True)
                    r.ev_done = torch.cuda.Event()
                    r.ev_done.record(self.down_stream)
                    self.copying.append(r)
        self.running = still
        rest = []
        for r in self.copying:
            if r.ev_done.query():
                r.t_done = now_fn()
                self.used -= r.fp
                r.df = r.out = None
                if not r.keep:
                    r.host_out = None
                    r.frame = None
                self.done.append(r)
            else:
                rest.append(r)
        self.copying = rest

    def busy(self):
        return bool(self.waiting or self.uploaded or self.running or self.copying)

    def step(self, now_fn):
        self._complete(now_fn)
        self._admit()
        self._launch()


def run(ctx, arrivals, make_frame, budget_bytes, split=0, max_batch=64, n_streams=2,
        keep_every=0, lookahead=32):
    """Serves `arrivals` (list of (t_seconds, recipe)) in real time.
    make_frame(recipe) builds the request's frame dict (host arrays); a
    producer thread builds them ahead of their arrival.  Requests whose index
    is a multiple of keep_every (if > 0) keep their inputs and output for
    checking.  Returns (server, wall seconds)."""
    srv = Server(ctx, budget_bytes, max_batch=max_batch, n_streams=n_streams)
    ready = collections.deque()
    lock = threading.Condition()
    stop = [False]

    def produce():
        for i, (t, recipe) in enumerate(arrivals):
            fr = make_frame(recipe)
            if not isinstance(fr["ac"], srv.torch.Tensor):
                fr = J.pin_frame(fr)  # inputs arrive in pinned host memory
            p = J.params(fr["xsize"], fr["ysize"], out_format=fr["out_format"], idct_split=split,
                         **fr["params"])
            keep = keep_every > 0 and i % keep_every == 0
            req = Request(i, t, fr, p, keep=keep)
            with lock:
                while len(ready) >= lookahead and not stop[0]:
                    lock.wait(0.01)
                if stop[0]:
                    return
                ready.append(req)
                lock.notify_all()

    prod = threading.Thread(target=produce, daemon=True)
    prod.start()
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    n = len(arrivals)
    try:
        while len(srv.done) < n:
            t = now()
            with lock:
                while ready and ready[0].t_arrival <= t:
                    srv.waiting.append(ready.popleft())
                    lock.notify_all()
            srv.step(now)
            if not srv.busy():
                time.sleep(0.0002)
    finally:
        with lock:
            stop[0] = True
            lock.notify_all()
        prod.join(timeout=5)
    srv.torch.cuda.synchronize()
    return srv, now()


def summarize(srv, wall):
    lat = np.array([(r.t_done - r.t_arrival) * 1e3 for r in srv.done])
    px = sum(r.params.xsize * r.params.ysize for r in srv.done)
    return dict(requests=len(srv.done), megapixels=round(px / 1e6, 3), wall_s=round(wall, 3),
                mp_per_s=round(px / 1e6 / wall, 3),
                latency_ms=dict(p50=round(float(np.percentile(lat, 50)), 3),
                                p90=round(float(np.percentile(lat, 90)), 3),
                                p99=round(float(np.percentile(lat, 99)), 3),
                                max=round(float(lat.max()), 3)),
                batches=srv.batches, mean_batch=round(float(np.mean(srv.batch_sizes)), 2),
                max_batch=int(max(srv.batch_sizes)), peak_budget_used_bytes=int(srv.peak_used),
                budget_bytes=int(srv.budget))
