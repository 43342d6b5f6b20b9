"""Serving driver: feeds a stream of Vecchia requests to the native engine
(include/vecchia.h, serve_*) in real time and reports latency percentiles and
throughput.  The engine (graph workers, HBM-arena admission, streams,
completion) is native; this module only marshals requests and results and
keeps the clock of the arrival process.

    python -m paper_2606_11402_amd.serve --requests 4096 --budget-gib 8

prints one JSON line: closed-loop capacity mu (requests/s), then the run at
lambda = 0.7 mu with p50/p99 latency (total and split into graph build, queue
and device time), points/s and peak HBM use.
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

from . import _lib

OP = {"forward": 0, "inverse": 1, "logdet": 2}


class Server:
    """One engine over an HBM arena of ``budget`` bytes (a torch tensor the
    server keeps alive), or a host-only mock engine."""

    def __init__(self, budget, n_streams=8, graph_workers=8, graph_threads=8, mock=False, device="cuda:0",
                 graph_device_bytes=0):
        """graph_device_bytes > 0: a second device buffer of that size, one
        slice per graph worker, in which the workers build the graphs of large
        requests on the GPU (serve_set_graph_device); the graphs are the
        same."""
        self._lib = _lib.load()
        self.mock = mock
        self.arena = None
        self.graph_buf = None
        ptr = None
        if not mock:
            import torch
            self.arena = torch.empty(int(budget), dtype=torch.uint8, device=device)
            ptr = ctypes.c_void_p(self.arena.data_ptr())
        h = ctypes.c_void_p()
        _lib.check(self._lib.serve_create(ptr, int(budget), n_streams, graph_workers, graph_threads, int(mock),
                                          ctypes.byref(h)), "serve_create")
        self._h = h
        self.meta = {}
        if graph_device_bytes and not mock:
            import torch
            self.graph_buf = torch.empty(int(graph_device_bytes), dtype=torch.uint8, device=device)
            _lib.check(self._lib.serve_set_graph_device(self._h, ctypes.c_void_p(self.graph_buf.data_ptr()),
                                                        int(graph_device_bytes)), "serve_set_graph_device")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.serve_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @staticmethod
    def request_bytes(n, k, n0=128):
        out = ctypes.c_size_t()
        _lib.check(_lib.load().serve_request_bytes(n, k, min(n0, n), ctypes.byref(out)), "serve_request_bytes")
        return out.value

    def submit(self, x, k, kind, sigma, ell, op, inp=None, nugget=0.0, n0=128):
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = x.shape[0]
        kern = _lib.KernelStruct(kind, sigma, ell, nugget)
        buf = None
        if op != "logdet":
            buf = np.ascontiguousarray(inp, dtype=np.float32)
        rid = ctypes.c_int64()
        _lib.check(self._lib.serve_submit(self._h, ctypes.c_void_p(x.ctypes.data), n, k, min(n0, n),
                                          ctypes.byref(kern), OP[op],
                                          ctypes.c_void_p(buf.ctypes.data) if buf is not None else None,
                                          ctypes.byref(rid)), "serve_submit")
        self.meta[rid.value] = (n, op)
        return rid.value

    def progress(self):
        n = ctypes.c_int32()
        _lib.check(self._lib.serve_progress(self._h, ctypes.byref(n)), "serve_progress")
        return n.value

    def take(self):
        rid = ctypes.c_int64()
        _lib.check(self._lib.serve_take(self._h, ctypes.byref(rid)), "serve_take")
        return rid.value

    def result(self, rid, release=True):
        n, op = self.meta[rid]
        out = np.empty(n, np.float32) if op != "logdet" else None
        ld = ctypes.c_double()
        times = (ctypes.c_double * 4)()
        rc = self._lib.serve_result(self._h, rid, ctypes.c_void_p(out.ctypes.data) if out is not None else None,
                                    ctypes.byref(ld), times)
        err = None if rc == 0 else _lib.VecchiaError(rc, self._lib.vecchia_last_error().decode())
        if release:
            self._lib.serve_release(self._h, rid)
            self.meta.pop(rid, None)
        if err is not None:
            raise err
        return (out if op != "logdet" else ld.value), list(times)

    def cancel(self, rid):
        _lib.check(self._lib.serve_cancel(self._h, rid), "serve_cancel")
        self.meta.pop(rid, None)
        self._lib.serve_release(self._h, rid)     # refused while a worker still builds it

    def stats(self):
        st = _lib.ServeStats()
        _lib.check(self._lib.serve_stats(self._h, ctypes.byref(st)), "serve_stats")
        return {name: getattr(st, name) for name, _ in st._fields_}

    def drain(self, timeout=600.0):
        """Progress until every submitted request has finished; returns
        {id: (result, times)} and releases them."""
        out = {}
        t0 = time.time()
        while len(out) < len(self.meta):
            self.progress()
            while True:
                rid = self.take()
                if not rid:
                    break
                out[rid] = self.result(rid, release=False)
            if time.time() - t0 > timeout:
                raise TimeoutError("requests still in flight after %.0fs" % timeout)
            time.sleep(0.0005)
        for rid in list(out):
            self._lib.serve_release(self._h, rid)
            self.meta.pop(rid, None)
        return out


def run_stream(requests, server, rate=None, kind=1, sigma=1.0, log=None, prefetch=48):
    """Submit requests at their arrival times (``rate`` rescales the Poisson
    stream to that many requests/s; None submits everything at t = 0, the
    closed-loop capacity run) and record latency = completion - arrival.
    Request inputs are generated ahead of the clock by a helper thread."""
    import queue
    import threading

    import workloads
    arrivals = [r.arrival for r in requests]
    if rate is not None and len(requests) > 1:
        scale = (len(requests) / rate) / max(arrivals[-1], 1e-9)
        arrivals = [a * scale for a in arrivals]
    q = queue.Queue(maxsize=prefetch)

    def producer():
        for r in requests:
            x = workloads.request_points(r)
            inp = None if r.op == "logdet" else workloads.request_xi(r)
            q.put((r, x, inp))

    th = threading.Thread(target=producer, daemon=True)
    th.start()
    t0 = time.perf_counter()
    ids, lat, parts, pts = {}, [], [], 0
    done = nxt = 0
    staged = None
    while done < len(requests):
        now = time.perf_counter() - t0
        while nxt < len(requests):
            if staged is None:
                try:
                    staged = q.get_nowait()
                except queue.Empty:
                    break
            t_arr = arrivals[nxt] if rate is not None else 0.0
            if t_arr > now:
                break
            r, x, inp = staged
            staged = None
            rid = server.submit(x, r.k, kind, sigma, r.ell, r.op, inp)
            ids[rid] = (nxt, t_arr)
            nxt += 1
        server.progress()
        while True:
            rid = server.take()
            if not rid:
                break
            i, t_arr = ids.pop(rid)
            _, times = server.result(rid)
            lat.append(time.perf_counter() - t0 - t_arr)
            parts.append(times)
            pts += requests[i].n
            done += 1
            if log and done % 512 == 0:
                log("%d/%d requests done, %.1fs" % (done, len(requests), time.perf_counter() - t0))
        time.sleep(0.0002)
    wall = time.perf_counter() - t0
    th.join()
    lat = np.array(lat)
    parts = np.array(parts)
    pc = lambda a, q_: float(np.percentile(a, q_))
    return {
        "requests": len(requests), "wall_s": wall, "req_per_s": len(requests) / wall, "points_per_s": pts / wall,
        "latency_p50_s": pc(lat, 50), "latency_p99_s": pc(lat, 99),
        "graph_p50_s": pc(parts[:, 0], 50), "graph_p99_s": pc(parts[:, 0], 99),
        "queue_p50_s": pc(parts[:, 1], 50), "queue_p99_s": pc(parts[:, 1], 99),
        "device_p50_s": pc(parts[:, 2], 50), "device_p99_s": pc(parts[:, 2], 99),
        "peak_hbm_bytes": server.stats()["peak_bytes"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=4096)
    ap.add_argument("--budget-gib", type=float, default=8.0)
    ap.add_argument("--streams", type=int, default=8)
    ap.add_argument("--workers", type=int, default=14)
    ap.add_argument("--load", type=float, nargs="*", default=[0.7])
    ap.add_argument("--graph-device-gib", type=float, default=3.0,
                    help="device buffer for graph builds on the GPU (0: every graph on the host)")
    args = ap.parse_args()
    gdev = int(args.graph_device_gib * (1 << 30))
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads
    log = lambda *a: print("[serve]", *a, file=sys.stderr, flush=True)
    reqs = workloads.request_stream(args.requests, rate=1.0)
    budget = int(args.budget_gib * (1 << 30))
    srv = Server(budget, n_streams=args.streams, graph_workers=args.workers, graph_device_bytes=gdev)
    log("closed loop (all requests at t=0)")
    closed = run_stream(reqs, srv, rate=None, log=log)
    mu = closed["req_per_s"]
    out = {"metric": "Vecchia serving: p50/p99 request latency and points/s", "mu_req_per_s": mu,
           "closed_loop": closed, "budget_bytes": budget, "streams": args.streams, "graph_workers": args.workers,
           "graph_device_bytes": gdev,
           "runs": []}
    for load in args.load:
        srv.close()
        srv = Server(budget, n_streams=args.streams, graph_workers=args.workers, graph_device_bytes=gdev)
        lam = load * mu
        log("open loop at lambda = %.1f req/s (%.2f mu)" % (lam, load))
        res = run_stream(reqs, srv, rate=lam, log=log)
        res["lambda_req_per_s"] = lam
        res["load"] = load
        out["runs"].append(res)
    srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
