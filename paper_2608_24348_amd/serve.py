"""Continuous-batching request loop for TGV and Poisson solves on one GPU.

Requests (a TGV run of a fixed number of steps, or a manufactured periodic
Poisson solve) arrive over time.  Each arrival is set up on the host
(``sem_setup``; workspace size known before any device memory is touched)
and waits in a FIFO until its workspace fits the HBM budget; admission binds
it (device geometry, initial condition or right-hand side).  Admitted
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
        self.ops = 0          # operator applications performed
        self.bytes = 0
        self.stats = []


class Server:
    """Runs a list of request specs (see inputs.request_stream) to completion."""

    def __init__(self, budget_bytes=None, max_batch=16, gmres_chunk=30, device="cuda:0", vel_tol=1e-6,
                 pres_tol=1e-4, poisson_tol=1e-8, keep_fields=False, policy="rr", tgv_steps=1, hsmg=1):
        import torch
        self.torch = torch
        self.device = device
        if budget_bytes is None:
            # blocks the caching allocator still holds from earlier work are
            # returned first, so the budget is the device's real free memory
            torch.cuda.empty_cache()
            free, _ = torch.cuda.mem_get_info(torch.device(device))
            budget_bytes = int(0.9 * free)
        self.budget = int(budget_bytes)
        self.max_batch = min(int(max_batch), 48)
        self.gmres_chunk = int(gmres_chunk)
        self.vel_tol = vel_tol          # TGV requests: the paper's absolute solver tolerances
        self.pres_tol = pres_tol
        self.poisson_tol = poisson_tol  # Poisson requests
        self.keep_fields = keep_fields
        # next batch key: "rr" round robin over keys with work, "oldest" the key
        # holding the longest-waiting active request
        if policy not in ("rr", "oldest"):
            raise ValueError("policy must be 'rr' or 'oldest'")
        self.policy = policy
        self.tgv_steps = max(1, int(tgv_steps))  # fluid steps per round of a TGV batch
        self.hsmg = 1 if hsmg else 0                # HSMG pressure preconditioner where a request allows it
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

    def _admit(self, r, now):
        torch = self.torch
        r.ctx.bind(self.device)
        self.used += r.bytes
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
            del f, rhs

    def _retire(self, r, now, status):
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
        self.used -= r.bytes
        r.ctx.close()
        r.ctx = None

    # ---------------------------------------------------------------- main loop
    def run(self, specs, log=None):
        reqs = [Request(s, self.hsmg) for s in sorted(specs, key=lambda s: s["arrival"])]
        pending = collections.deque(reqs)
        waiting = collections.deque()
        active = collections.OrderedDict()
        keys_rr = collections.deque()
        t0 = time.perf_counter()
        done = []
        rounds = 0
        while pending or waiting or any(active.values()):
            now = time.perf_counter() - t0
            while pending and pending[0].spec["arrival"] <= now:
                r = pending.popleft()
                r.t_arrival = r.spec["arrival"]
                self._setup(r)
                waiting.append(r)
            # FIFO admission under the HBM budget
            while waiting and self.used + waiting[0].bytes <= self.budget:
                r = waiting.popleft()
                self._admit(r, time.perf_counter() - t0)
                active.setdefault(r.key, []).append(r)
                if r.key not in keys_rr:
                    keys_rr.append(r.key)
            if not any(active.values()):
                if waiting and self.used == 0:
                    # larger than the whole budget: reject instead of deadlocking
                    r = waiting.popleft()
                    r.t_done = time.perf_counter() - t0
                    r.status = "rejected"
                    r.ctx.close()
                    done.append(r)
                    continue
                if pending:
                    time.sleep(max(0.0, min(0.05, pending[0].spec["arrival"] - (time.perf_counter() - t0))))
                continue
            if self.policy == "oldest":
                key = min((k for k, v in active.items() if v), key=lambda k: active[k][0].t_arrival)
            else:
                # next batch key with work (round robin)
                while not active.get(keys_rr[0]):
                    keys_rr.rotate(-1)
                key = keys_rr[0]
                keys_rr.rotate(-1)
            batch = active[key][:self.max_batch]
            ctxs = [r.ctx for r in batch]
            rounds += 1
            if key[2] == "tgv":
                # as many steps as the batch's requests all still need, at most tgv_steps
                k = min([self.tgv_steps] + [r.spec["steps"] - r.steps_done for r in batch])
                st = sem.fluid_step(ctxs, k)
                now = time.perf_counter() - t0
                for r, ss in zip(batch, st):
                    bad = 0
                    for s in ss:
                        r.steps_done += 1
                        r.stats.append(s)
                        r.ops += sum(s["vit"]) + s["pit"] + (6 if r.spec["tier"] != "fp64" else 3) + 1
                        bad = bad or s["status"]
                    s = {"status": bad}
                    if s["status"] != 0 or r.steps_done >= r.spec["steps"]:
                        self._retire(r, now, "ok" if s["status"] == 0 else "status%d" % s["status"])
                        active[key].remove(r)
                        done.append(r)
            else:
                flags = sem.poisson_advance(ctxs, self.gmres_chunk)
                now = time.perf_counter() - t0
                for r, a in zip(batch, flags):
                    if not a:
                        self._retire(r, now, "ok")
                        st = r.result["stats"]
                        r.ops += st["iters"] + 2
                        if st["status"] != 0:
                            r.status = "status%d" % st["status"]
                        active[key].remove(r)
                        done.append(r)
            if log and rounds % 50 == 0:
                log("round %d t=%.2fs active=%d waiting=%d done=%d used=%.1f GB"
                    % (rounds, now, sum(len(v) for v in active.values()), len(waiting), len(done), self.used / 1e9))
        makespan = time.perf_counter() - t0
        return done, makespan


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
    args = ap.parse_args()
    sem.load()
    res = measure(args.requests, args.seed, tuple(float(x) for x in args.loads.split(",")), args.max_batch,
                  log=lambda m: print(m, file=sys.stderr, flush=True), hsmg=args.hsmg)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
