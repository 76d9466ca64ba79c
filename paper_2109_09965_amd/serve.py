"""Continuous-batching steady-solve server over the pool API.

Requests (a prepared mesh, its free stream and gas parameters, a
tolerance) arrive over time.  The server keeps one pool per dimension, each
with a fixed capacity carved out of an HBM budget, and each on its own HIP
stream so the two pools' work overlaps on the device.  Each pool runs its
own sequence of epochs: whenever its previous epoch has finished (an event
on its stream), the server reads that epoch's per-case Res history, retires
cases that converged (or stalled at their precision's floor, or hit the
cycle cap: their state is downloaded to the host and their ranges
released), admits waiting requests of its dimension in arrival order while
their mesh fits into free ranges (the pool's HBM footprint), and replays a
captured graph of ``epoch_cycles`` cycles of every admitted case.  No pool
waits for another's epoch, so host work for one pool overlaps the other's
cycles.  A case gives bitwise the same state in the mix as alone after the
same number of cycles.

Time-to-steady runs from a request's arrival to its converged state on the
host; queue wait (arrival to admission) and service (admission to done) are
reported with it.
"""
import dataclasses
import time

import numpy as np

from . import FP64, Batch, Params

# Faces, Gauss points and boundary faces reserved per cell of capacity:
# upper bounds over the trace's meshes (cylinder O-grids: 1.5 faces and 3
# Gauss points per cell, boundary faces 1/n_r per cell; hybrid sphere
# O-grids: 2 (tets) to 3 (hexes) faces and 6 to 12 Gauss points per cell,
# boundary faces up to a fifth of the cells on coarse grids).  They cost
# far less than a cell (see entity_bytes), so the margins are cheap.
ENTITY_RATIOS = {2: (1.0, 1.6, 3.2, 0.25), 3: (1.0, 3.0, 12.0, 0.25)}


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the trace
    mesh: object              # paper_2109_09965_amd.Mesh (prepared by the client)
    params: Params
    W0: np.ndarray
    dW0: np.ndarray
    tol: float
    # filled in by the server
    admitted: float = None
    done: float = None
    cycles: int = 0           # all cycles the case ran
    cycles_fp64: int = 0      # of them, cycles in an FP64 finishing pool
    res_first: float = None
    res_last: float = None
    best: float = np.inf
    best_at: int = 0
    status: str = "waiting"
    W: np.ndarray = None
    dW: np.ndarray = None
    slot: int = None
    key: tuple = None         # (pool kind, dim) the case runs in


def entity_bytes(dim, precision):
    """Pool bytes per cell, face, Gauss point and boundary face."""
    import ctypes as C
    from . import _PoolDesc, _check, lib
    L = lib()

    def nbytes(*caps):
        q = _PoolDesc(dim, precision, 1, *caps, 6, 2, 0, 0)
        h = C.c_void_p()
        _check(L.cgks_pool_create(C.byref(q), C.byref(h)), "cgks_pool_create")
        nb = C.c_size_t()
        _check(L.cgks_batch_query(h, C.byref(nb)), "cgks_batch_query")
        L.cgks_batch_destroy(h)
        return nb.value

    one = 1 << 20
    base = nbytes(one, one, one, one)
    out = []
    for k in range(4):
        caps = [one] * 4
        caps[k] = 2 * one
        out.append((nbytes(*caps) - base) / one)
    return out


def caps_for_budget(dim, precision, budget_bytes):
    """Entity capacities of a pool that fits budget_bytes, proportioned for
    meshes of the given dimension."""
    per = entity_bytes(dim, precision)
    ratios = ENTITY_RATIOS[dim]
    cells = int(budget_bytes / sum(p * r for p, r in zip(per, ratios)))
    return [max(1, int(cells * r)) for r in ratios]


class Server:
    """max_resident[dim]: cells a pool may hold at once beyond its first
    case.  A few hundred thousand cells already fill the GPU, so letting more
    in only time-shares it (every case then advances more slowly); small
    cases still batch up to the cap.  None = bounded by memory alone.

    finish_fp64 (mixed precisions): a case whose Res stops improving (by 1 %
    over promote_after cycles) before reaching its tolerance has met the FP32
    floor; it moves, state and gradients, into an FP64 pool of its dimension
    and finishes there (admitted ahead of new arrivals)."""

    def __init__(self, budget_bytes, precision=FP64, max_cases=64, epoch_cycles=8, max_cycles=4000,
                 stall_cycles=400, share_3d=0.75, max_resident=None, finish_fp64=False, fp64_share=0.3,
                 promote_after=100):
        import torch
        self.precision = precision
        self.epoch = epoch_cycles
        self.max_cycles = max_cycles
        self.stall = stall_cycles
        self.promote_after = promote_after
        self.finish = finish_fp64 and precision != FP64
        kinds = [("run", precision, 1.0 - fp64_share if self.finish else 1.0)]
        if self.finish:
            kinds.append(("fp64", FP64, fp64_share))
        self.pools, self.streams = {}, {}
        for kind, prec, share in kinds:
            for dim, dshare in ((2, 1.0 - share_3d), (3, share_3d)):
                key = (kind, dim)
                caps = caps_for_budget(dim, prec, share * dshare * budget_bytes)
                st = torch.cuda.Stream()
                self.streams[key] = st
                self.pools[key] = Batch.pool(dim, max_cases, *caps, precision=prec, stream=st)
        self.max_resident = max_resident or {}
        self.live = {k: {} for k in self.pools}       # slot -> Request
        self.dirty = {k: True for k in self.pools}    # membership changed: capture again
        self.to_finish = []                           # promoted cases waiting for an FP64 slot
        self.inflight = {}                            # pool -> (event, Res history, cell-updates) of its epoch

    def _admit(self, key, req, W, dW):
        dim = key[1]
        cap = self.max_resident.get(dim)
        resident = sum(r.mesh.n_cell for r in self.live[key].values())
        if cap is not None and self.live[key] and resident + req.mesh.n_cell > cap:
            return False
        pool = self.pools[key]
        slot = pool.admit(req.mesh, req.params)
        if slot is None:
            return False
        pool.upload(slot, W, dW)
        req.slot, req.key = slot, key
        self.live[key][slot] = req
        self.dirty[key] = True
        return True

    def try_admit(self, req, now):
        if not self._admit(("run", req.mesh.dim), req, req.W0, req.dW0):
            return False
        req.admitted, req.status = now, "running"
        return True

    def launch(self, key):
        """Start one epoch of the pool on its stream (capturing its graph
        again if its membership changed)."""
        import torch
        pool, st = self.pools[key], self.streams[key]
        with torch.cuda.stream(st):
            if self.dirty[key]:
                pool.graph_create(self.epoch)
                self.dirty[key] = False
            h = torch.zeros(self.epoch * pool.n_case, dtype=torch.float64, device="cuda")
            pool.graph_launch(h)
            ev = torch.cuda.Event()
            ev.record(st)
        work = self.epoch * sum(r.mesh.n_cell for r in self.live[key].values())
        self.inflight[key] = (ev, h, work)

    def collect(self, key, now_fn):
        """Wait for the pool's epoch, retire its finished cases; returns
        (cell-updates of the epoch, requests finished)."""
        ev, h, work = self.inflight.pop(key)
        ev.synchronize()
        H = h.cpu().numpy().reshape(self.epoch, -1)
        return work, self.retire({key: H}, now_fn)

    def retire(self, hist, now_fn):
        done = []
        for key, H in hist.items():
            pool = self.pools[key]
            promote_ok = self.finish and key[0] == "run"
            for slot, req in list(self.live[key].items()):
                finished = None
                for j in range(self.epoch):
                    r = float(H[j, slot])
                    req.cycles += 1
                    if key[0] == "fp64":
                        req.cycles_fp64 += 1
                    if req.res_first is None:
                        req.res_first = r
                    req.res_last = r
                    if r < 0.99 * req.best:
                        req.best, req.best_at = r, req.cycles
                    if finished is not None:
                        continue
                    if not np.isfinite(r):
                        finished = "nonphysical"
                    elif r <= req.tol:
                        finished = "converged"
                    elif promote_ok and req.cycles - req.best_at >= self.promote_after:
                        finished = "promote"
                    elif req.cycles - req.best_at >= self.stall:
                        finished = "stalled"
                    elif req.cycles >= self.max_cycles:
                        finished = "max_cycles"
                # the state after the epoch's last cycle (req.cycles counts
                # every cycle the case ran)
                if finished:
                    req.W, req.dW = pool.download(slot)
                    pool.release(slot)
                    del self.live[key][slot]
                    self.dirty[key] = True
                    if finished == "promote":
                        req.status, req.best, req.best_at = "finishing", np.inf, req.cycles
                        self.to_finish.append(req)
                        continue
                    req.status, req.done = finished, now_fn()
                    done.append(req)
        return done

    def run(self, requests, log=None):
        """Serve a trace (requests sorted by arrival); returns a summary."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        waiting, nxt, finished = [], 0, []
        work = 0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        while len(finished) < len(reqs):
            t = now()
            while nxt < len(reqs) and reqs[nxt].arrival <= t:
                waiting.append(reqs[nxt])
                nxt += 1
            # pools whose epoch has finished: retire
            progressed = False
            for key in list(self.inflight):
                if self.inflight[key][0].query():
                    w, done = self.collect(key, now)
                    work += w
                    finished += done
                    progressed = True
                    if log:
                        for r in done:
                            log(r)
            # admissions go into pools between their epochs only; promoted
            # cases first (they hold no memory while they wait)
            for req in list(self.to_finish):
                key = ("fp64", req.mesh.dim)
                if key in self.inflight:
                    continue
                if self._admit(key, req, req.W, req.dW):
                    self.to_finish.remove(req)
                elif not self.live[key]:
                    # no room even in the empty FP64 pool: keep the FP32 result
                    req.status, req.done = "stalled", now()
                    self.to_finish.remove(req)
                    finished.append(req)
            # arrival order per dimension: a request that does not fit blocks
            # later ones of its dimension (no starvation of large cases)
            blocked = set()
            for req in list(waiting):
                d = req.mesh.dim
                if d in blocked:
                    continue
                if ("run", d) in self.inflight:
                    blocked.add(d)
                    continue
                if self.try_admit(req, t):
                    waiting.remove(req)
                elif not self.live[("run", d)]:
                    # does not fit even into the empty pool: never will
                    req.status, req.admitted, req.done = "rejected", t, t
                    waiting.remove(req)
                    finished.append(req)
                else:
                    blocked.add(d)
            # every idle pool with cases starts its next epoch
            for key in self.pools:
                if key not in self.inflight and self.live[key]:
                    self.launch(key)
                    progressed = True
            if not self.inflight:
                if nxt < len(reqs) and not self.to_finish:
                    time.sleep(max(0.0, min(0.01, reqs[nxt].arrival - now())))
                continue
            if not progressed:
                time.sleep(2e-4)   # poll the running epochs
        makespan = now()
        return summarize(finished, work, makespan)


def summarize(finished, work, makespan):
    """Aggregate throughput over all requests; p50/p99 time-to-steady,
    queue wait and service time over the converged requests only (a
    request that stalled, diverged, went non-physical or hit the cycle cap
    has no time-to-steady); the other outcomes are counted beside them."""
    conv = [r for r in finished if r.status == "converged"]
    status = {}
    for r in finished:
        status[r.status] = status.get(r.status, 0) + 1

    def pct(vals, q):
        return float(np.percentile(vals, q)) if len(vals) else None
    tts = np.array([r.done - r.arrival for r in conv])
    wait = np.array([r.admitted - r.arrival for r in conv])
    svc = np.array([r.done - r.admitted for r in conv])
    return dict(requests=len(finished), converged=len(conv), not_converged=len(finished) - len(conv),
                makespan_s=makespan, cell_updates=int(work),
                fp64_finishing_cycles=int(sum(r.cycles_fp64 for r in finished)),
                cell_updates_per_s=work / makespan if makespan > 0 else 0.0,
                p50_time_to_steady_s=pct(tts, 50), p99_time_to_steady_s=pct(tts, 99),
                p50_queue_wait_s=pct(wait, 50), p99_queue_wait_s=pct(wait, 99),
                p50_service_s=pct(svc, 50), p99_service_s=pct(svc, 99),
                status=status)
