"""Continuous-batching request loop for TGV and Poisson solves on one GPU.

Requests (a TGV run of a fixed number of steps, or a manufactured periodic
Poisson solve) arrive over time.  Each arrival is set up on the host
(``sem_setup``; workspace size known before any device memory is touched)
and waits in a FIFO until its workspace fits in the server's arena (the HBM
budget, one device allocation, first fit); admission binds it there
(device geometry, initial condition or right-hand side) on an admission
stream, then hands it to the stream of the worker that owns its key.  Admitted
requests are grouped by batch key (polynomial order, precision tier, kind,
pressure preconditioner: HSMG where the request allows it, else Jacobi);
every round the loop takes the next key with work, forms a batch of up to
``max_batch`` requests and runs one unit of work for all of them in single
batched launches: one fluid time step for TGV requests, or one chunk of
GMRES iterations for Poisson requests.  Requests finish independently and
leave; waiting requests are admitted as memory frees up, so requests that
arrive while others run join the next round (continuous batching).  All
solver state lives on the device per request and every reduction is per
request in fixed order, so a request's result does not depend on what it was
batched with.

Latency is completion minus arrival (wall clock of this process); aggregate
GDOF/s counts E*lx^3 per operator application.
"""
import collections
import math
import time

import numpy as np

from . import sem


def _hsmg_ok(spec):
    """the HSMG pressure preconditioner needs order >= 4 and 2..64 elements per direction"""
    return spec["N"] >= 4 and all(2 <= n <= 64 for n in spec["nel"])


def _key(spec, hsmg=0):
    return (spec["N"] + 1, spec["tier"], spec["kind"], 1 if hsmg and _hsmg_ok(spec) else 0)


class Request:
    def __init__(self, spec, hsmg=0):
        self.spec = spec
        self.kind = spec["kind"]
        self.key = _key(spec, hsmg)
        self.ctx = None
        self.steps_done = 0
        self.t_arrival = None
        self.t_admit = None
        self.t_done = None
        self.status = None
        self.result = None
        self.slot = None      # (offset, bytes) of its workspace in the arena
        self.ops = 0          # operator applications performed
        self.bytes = 0
        self.ctx_points = 0
        self.stats = []


class _Arena:
    """Request workspaces carved out of one device buffer: first fit over a
    sorted free list, 256-byte granules, freed ranges merged with their
    neighbours.  One allocation per server run instead of one per request."""

    G = 256

    def __init__(self, torch, nbytes, device, buf=None):
        self.size = max(self.G, nbytes // self.G * self.G)
        if buf is None:
            buf = torch.empty(self.size + self.G, dtype=torch.uint8, device=device)
        assert buf.numel() >= self.size + self.G
        self.buf = buf
        self.base = (-self.buf.data_ptr()) % self.G   # first 256-byte aligned offset
        self.free = [[0, self.size]]                   # [offset, bytes], sorted, disjoint

    def alloc(self, nbytes):
        n = -(-nbytes // self.G) * self.G
        for i, (o, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    del self.free[i]
                else:
                    self.free[i] = [o + n, sz - n]
                return o, n
        return None

    def view(self, off, n):
        return self.buf[self.base + off:self.base + off + n]

    def release(self, off, n):
        i = 0
        while i < len(self.free) and self.free[i][0] < off:
            i += 1
        self.free.insert(i, [off, n])
        if i + 1 < len(self.free) and off + n == self.free[i + 1][0]:
            self.free[i][1] += self.free[i + 1][1]
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:
            self.free[i - 1][1] += self.free[i][1]
            del self.free[i]

    def empty(self):
        return self.free == [[0, self.size]]


class _Worker:
    """One host thread and one HIP stream (default priority).  It owns the batch
    keys assigned to it and runs their rounds one after another; the workers
    run concurrently, so batches of different keys overlap on the device."""

    def __init__(self, idx, stream):
        self.idx = idx
        self.stream = stream
        self.keys = collections.deque()   # keys owned, round-robin order
        self.load = 0                     # local points of its active requests


class Server:
    """Runs a list of request specs (see inputs.request_stream) to completion."""

    def __init__(self, budget_bytes=None, max_batch=16, gmres_chunk=30, device="cuda:0", vel_tol=1e-6,
                 pres_tol=1e-4, poisson_tol=1e-8, keep_fields=False, policy="rr", tgv_steps=1, hsmg=1,
                 streams=4, graph=True):
        import torch
        self.torch = torch
        self.device = device
        if budget_bytes is None:
            # blocks the caching allocator still holds from earlier work are
            # returned first, so the budget is the device's real free memory
            # (plus the arena an earlier server of this process left)
            torch.cuda.empty_cache()
            free, _ = torch.cuda.mem_get_info(torch.device(device))
            budget_bytes = int(0.9 * (free + _arena_held(device)))
        self.budget = int(budget_bytes)
        self.max_batch = min(int(max_batch), 48)
        self.gmres_chunk = int(gmres_chunk)
        self.vel_tol = vel_tol          # TGV requests: the paper's absolute solver tolerances
        self.pres_tol = pres_tol
        self.poisson_tol = poisson_tol  # Poisson requests
        self.keep_fields = keep_fields
        # next batch key of a worker: "rr" round robin over its keys with work,
        # "oldest" the key holding its longest-waiting active request
        if policy not in ("rr", "oldest"):
            raise ValueError("policy must be 'rr' or 'oldest'")
        self.policy = policy
        self.tgv_steps = max(1, int(tgv_steps))  # fluid steps per round of a TGV batch
        self.hsmg = 1 if hsmg else 0                # HSMG pressure preconditioner where a request allows it
        self.nstreams = max(1, min(int(streams), 4))
        self.graph = bool(graph)                    # TGV steps replayed as HIP graphs
        self.used = 0

    # ---------------------------------------------------------------- request life cycle
    def _setup(self, r):
        s = r.spec
        mode = sem.MODE_FLUID if r.kind == "tgv" else sem.MODE_POISSON
        ptol = self.pres_tol if r.kind == "tgv" else self.poisson_tol
        flow = sem.flow_desc(mode=mode, nu=1.0 / s["Re"], dt=s["dt"], vel_tol=self.vel_tol, pres_tol=ptol,
                             pres_maxit=3000, hsmg=r.key[3])
        r.ctx = sem.Context(sem.mesh_desc(s["nel"], s["N"]), flow, sem.tier(s["tier"]), device=self.device,
                            bind=False)
        r.bytes = r.ctx.bytes + 256

    def _admit(self, r, now, w):
        torch = self.torch
        # geometry and rhs are made on the admission stream, in the request's
        # slice of the arena, under the library's host lock (no worker captures
        # a step graph meanwhile); once that stream is done the request moves
        # to the stream of the worker that owns its key, so admission never
        # waits for a worker's queued steps
        adm = self.adm_stream
        with sem.host_lock(), torch.cuda.stream(adm):
            r.ctx.bind(self.device, stream=adm, workspace=self.arena.view(*r.slot))
            r.t_admit = now
            if r.kind == "poisson":
                # manufactured rhs: f = 3 sin x sin y sin z + noise (seeded N(0,1) per local point)
                f = r.ctx.node_field(3, 3.0)
                g = torch.Generator(device=self.device)
                g.manual_seed(int(r.spec["noise_seed"]))
                f.add_(torch.randn(r.ctx.np, dtype=torch.float64, device=self.device, generator=g),
                       alpha=float(r.spec["noise"]))
                rhs = r.ctx.mass(f, assemble=True)
                sem.poisson_begin([r.ctx], [rhs])
            adm.synchronize()
            if r.kind == "poisson":
                del f, rhs
            r.ctx.set_stream(w.stream)

    def _retire(self, r, now, status):
        with sem.host_lock():
            self._retire_locked(r, now, status)

    def _retire_locked(self, r, now, status):
        r.t_done = now
        r.status = status
        if self.keep_fields:
            if r.kind == "tgv":
                r.result = {"u": r.ctx.velocity(), "p": r.ctx.pressure()}
            else:
                sol = self.torch.empty(r.ctx.np, dtype=self.torch.float64, device=self.device)
                st = sem.poisson_finish(r.ctx, sol)
                r.result = {"p": sol.cpu().numpy(), "stats": st}
        elif r.kind == "poisson":
            r.result = {"stats": sem.poisson_finish(r.ctx, None)}
        r.ctx.close()
        r.ctx = None

    # ---------------------------------------------------------------- one round of a worker
    def _round(self, key, batch):
        """One unit of work for a batch (runs without the lock); returns the
        requests that finished, each with its status."""
        ctxs = [r.ctx for r in batch]
        out = []
        if key[2] == "tgv":
            # as many steps as the batch's requests all still need, at most tgv_steps
            k = min([self.tgv_steps] + [r.spec["steps"] - r.steps_done for r in batch])
            st = sem.fluid_step(ctxs, k, graph=self.graph)
            for r, ss in zip(batch, st):
                bad = 0
                for s in ss:
                    r.steps_done += 1
                    r.stats.append(s)
                    r.ops += sum(s["vit"]) + s["pit"] + (6 if r.spec["tier"] != "fp64" else 3) + 1
                    bad = bad or s["status"]
                if bad != 0 or r.steps_done >= r.spec["steps"]:
                    out.append((r, "ok" if bad == 0 else "status%d" % bad))
        else:
            flags = sem.poisson_advance(ctxs, self.gmres_chunk)
            for r, a in zip(batch, flags):
                if not a:
                    out.append((r, "ok"))
        return out

    # ---------------------------------------------------------------- main loop
    def run(self, specs, log=None):
        import threading
        torch = self.torch
        reqs = [Request(s, self.hsmg) for s in sorted(specs, key=lambda s: s["arrival"])]
        pending = collections.deque(reqs)
        waiting = collections.deque()
        active = collections.OrderedDict()   # key -> admitted requests
        owner = {}                           # key -> worker
        workers = [_Worker(i, _stream(torch, self.device, i)) for i in range(self.nstreams)]
        self.adm_stream = _stream(torch, self.device, "admission")
        self.arena = _Arena(torch, self.budget, self.device, _arena_buffer(torch, self.device, self.budget))
        cv = threading.Condition()
        done = []
        state = {"rounds": 0, "error": None, "stop": False}
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        def worker_loop(w):
            try:
                while True:
                    with cv:
                        while not state["stop"] and not any(active.get(k) for k in w.keys):
                            cv.wait()
                        if state["stop"]:
                            return
                        keys = [k for k in w.keys if active.get(k)]
                        if self.policy == "oldest":
                            key = min(keys, key=lambda k: active[k][0].t_arrival)
                        else:
                            while not active.get(w.keys[0]):
                                w.keys.rotate(-1)
                            key = w.keys[0]
                            w.keys.rotate(-1)
                        batch = active[key][:self.max_batch]
                        state["rounds"] += 1
                        rnd = state["rounds"]
                    finished = self._round(key, batch)
                    now = clock()
                    for r, status in finished:
                        self._retire(r, now, status)
                        if r.kind == "poisson":
                            st = r.result["stats"]
                            r.ops += st["iters"] + 2
                            if st["status"] != 0:
                                r.status = "status%d" % st["status"]
                    with cv:
                        for r, _ in finished:
                            active[key].remove(r)
                            # the request's work is complete and its context closed
                            self.arena.release(*r.slot)
                            r.slot = None
                            self.used -= r.bytes
                            w.load -= r.ctx_points
                            done.append(r)
                        cv.notify_all()
                    if log and rnd % 50 == 0:
                        log("round %d t=%.2fs active=%d waiting=%d done=%d used=%.1f GB"
                            % (rnd, now, sum(len(v) for v in active.values()), len(waiting), len(done),
                               self.used / 1e9))
            except BaseException as e:  # surface worker failures in the main thread
                with cv:
                    state["error"] = e
                    state["stop"] = True
                    cv.notify_all()

        threads = [threading.Thread(target=worker_loop, args=(w,), daemon=True) for w in workers]
        for th in threads:
            th.start()
        try:
            while True:
                with cv:
                    if state["error"] is not None:
                        raise state["error"]
                    if not pending and not waiting and not any(active.values()):
                        break
                now = clock()
                while pending and pending[0].spec["arrival"] <= now:
                    r = pending.popleft()
                    r.t_arrival = r.spec["arrival"]
                    self._setup(r)
                    waiting.append(r)
                # FIFO admission under the HBM budget
                admitted = False
                while waiting:
                    with cv:
                        slot = self.arena.alloc(waiting[0].bytes)
                        idle = self.arena.empty() and not any(active.values())
                    r = waiting[0]
                    if slot is None:
                        if idle:
                            # larger than the whole budget: reject instead of deadlocking
                            waiting.popleft()
                            r.t_done = clock()
                            r.status = "rejected"
                            with sem.host_lock():
                                r.ctx.close()
                            with cv:
                                done.append(r)
                            continue
                        break
                    waiting.popleft()
                    r.slot = slot
                    with cv:
                        w = owner.get(r.key)
                        if w is None or not active.get(r.key):
                            # a new (or drained) key goes to the least loaded worker
                            if w is not None and r.key in w.keys:
                                w.keys.remove(r.key)
                            w = min(workers, key=lambda x: x.load)
                            owner[r.key] = w
                            w.keys.append(r.key)
                        self.used += r.bytes
                        r.ctx_points = r.ctx.np
                        w.load += r.ctx_points
                    self._admit(r, clock(), w)
                    with cv:
                        active.setdefault(r.key, []).append(r)
                        cv.notify_all()
                    admitted = True
                if admitted:
                    continue
                # sleep until the next arrival or until a worker retires a request
                with cv:
                    if state["error"] is None and (pending or waiting):
                        wait = 0.05 if not pending else max(0.0, min(0.05, pending[0].spec["arrival"] - clock()))
                        cv.wait(timeout=wait)
                    elif state["error"] is None and any(active.values()):
                        cv.wait(timeout=0.05)
        finally:
            with cv:
                state["stop"] = True
                cv.notify_all()
            for th in threads:
                th.join()
            torch.cuda.synchronize()
            self.arena = None
        makespan = clock()
        return done, makespan


# streams are kept for the process: a server made per measurement reuses them
# instead of creating (and leaking) hardware-queue slots every time
_STREAMS = {}
# the workspace arena is kept for the process too (one device allocation of
# the budget, reused by later servers; release_arena gives it back)
_ARENAS = {}


def _arena_held(device):
    buf = _ARENAS.get(str(device))
    return 0 if buf is None else buf.numel()


def _arena_buffer(torch, device, nbytes):
    need = nbytes + _Arena.G
    buf = _ARENAS.get(str(device))
    if buf is None or buf.numel() < need:
        _ARENAS.pop(str(device), None)
        buf = None
        torch.cuda.empty_cache()
        buf = torch.empty(need, dtype=torch.uint8, device=device)
        _ARENAS[str(device)] = buf
    return buf


def release_arena(device="cuda:0"):
    """Give the servers' workspace arena of this process back to the device."""
    import torch
    if _ARENAS.pop(str(device), None) is not None:
        torch.cuda.empty_cache()


def _stream(torch, device, tag):
    key = (str(device), tag)
    if key not in _STREAMS:
        _STREAMS[key] = torch.cuda.Stream(device=device)
    return _STREAMS[key]


def summarize(done, makespan):
    lat = np.array([r.t_done - r.t_arrival for r in done if r.status == "ok"])
    gdof = sum(r.ops * (r.spec["nel"][0] * r.spec["nel"][1] * r.spec["nel"][2] * (r.spec["N"] + 1) ** 3)
               for r in done if r.status == "ok")
    out = {"requests": len(done), "ok": int(sum(r.status == "ok" for r in done)),
           "rejected": int(sum(r.status == "rejected" for r in done)), "makespan_s": makespan,
           "requests_per_s": len(done) / makespan, "gdof_per_s": gdof / makespan / 1e9}
    if len(lat):
        out.update({"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                    "mean_s": float(lat.mean()), "max_s": float(lat.max())})
        # the tail: the three slowest requests, with their wait for admission
        # and their time from admission to completion
        ok = sorted((r for r in done if r.status == "ok"), key=lambda r: r.t_done - r.t_arrival)[-3:]
        out["slowest"] = [{"kind": r.spec["kind"], "nel": list(r.spec["nel"]), "N": r.spec["N"], "tier": r.spec["tier"],
                           "latency_s": r.t_done - r.t_arrival, "admit_wait_s": r.t_admit - r.t_arrival,
                           "service_s": r.t_done - r.t_admit} for r in reversed(ok)]
    return out


def measure(n_requests=256, seed=24348, loads=(0.4, 0.7, 1.0), max_batch=16, log=None, **server_kw):
    """Serving measurement: a burst of the whole stream (all requests at t = 0)
    gives the saturated request rate; the same stream is then replayed with
    Poisson arrivals at each fraction of that rate."""
    from . import inputs
    out = {"requests": n_requests, "seed": seed}
    burst = inputs.request_stream(n_requests=n_requests, qps=1e12, seed=seed)
    done, ms = Server(max_batch=max_batch, **server_kw).run(burst, log=log)
    sat = summarize(done, ms)
    out["saturated"] = sat
    for f in loads:
        qps = f * sat["requests_per_s"]
        specs = inputs.request_stream(n_requests=n_requests, qps=qps, seed=seed)
        done, ms = Server(max_batch=max_batch, **server_kw).run(specs, log=log)
        out["load_%.1f" % f] = dict(summarize(done, ms), qps=qps)
    release_arena(server_kw.get("device", "cuda:0"))
    return out


def main():
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="Serve a seeded stream of TGV and Poisson requests on one GPU")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--seed", type=int, default=24348)
    ap.add_argument("--loads", default="0.4,0.7,1.0", help="fractions of the saturated request rate")
    ap.add_argument("--max-batch", type=int, default=16)
    ap.add_argument("--hsmg", type=int, default=1, choices=[0, 1],
                    help="HSMG pressure preconditioner where a request allows it (1), Jacobi everywhere (0)")
    ap.add_argument("--streams", type=int, default=4, help="worker streams (host threads), 1..4")
    ap.add_argument("--graph", type=int, default=1, choices=[0, 1], help="TGV steps replayed as HIP graphs")
    args = ap.parse_args()
    sem.load()
    res = measure(args.requests, args.seed, tuple(float(x) for x in args.loads.split(",")), args.max_batch,
                  log=lambda m: print(m, file=sys.stderr, flush=True), hsmg=args.hsmg, streams=args.streams,
                  graph=bool(args.graph))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
