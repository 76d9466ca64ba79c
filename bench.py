"""Benchmark: cell-updates/s of the p-multigrid CGKS cycle on one MI355X.

One step = one two-level cycle (S2O4 high-order step with Gauss-Green
gradient update, high-order residual, KFVS forcing, 6 implicit steps of 2
multicolour point-relaxation sweeps, prolongation, Res) on every cell of the
workload.  Default workload: 3-D hybrid sphere O-grid on a cubed-sphere
surface (6 x 28 x 28 quads, 40 layers: 20 hex, 10 prism, 10 tet; 470,400
cells), Ma 0.25, Re 100, Pr 0.72, no-slip adiabatic wall, FP64.  Inputs are resident on the device
before the timed region.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# MI355X vector peaks: FP64 78.6 TFLOP/s (256 CUs x 2.4 GHz x 64 FMA per
# clock).  The published FP32 figure, 157.3, counts packed FP32 (two
# operations per lane per instruction); the library is compiled with
# packed FP32 off, so an FP32 lane operation issues at the FP64 rate and the FP32
# kernels are priced at 78.6 as well.
VALU_PEAK_TFLOPS = {"fp64": 78.6, "mixed32": 78.6, "mixed32_r64": 78.6}
FP32_PACKED_PEAK_TFLOPS = 157.3

# Floating-point operations of the high-order flux kernel per Gauss point
# (FMA = 2), from the VALU instruction counters of one launch on the
# sphere workload (SQ_INSTS_VALU_{FMA,MUL,ADD,TRANS}_F64 resp. _F32, x 64
# lanes), charged to the lanes that carry a Gauss point.
FLUX_FLOP_PER_GP = {"fp64": 1514.9, "mixed32": 1386.0, "mixed32_r64": (2 * 1386.0 + 1514.9) / 3.0}

# HBM bytes per launch from rocprofv3 FETCH_SIZE (x 2.0) and WRITE_SIZE
# (x 1.0) on the sphere workload, each factor from a plain device copy of
# known size.  Valid only for the kernel source they were taken on (its
# SHA-256); any other source reports null.
PROFILED_KERNELS_SHA256 = "587da4672ae8271f13d071f2ebb32955ec7c8fdf19014b179ced2c7d0fa34b88"
PROFILED_TRAFFIC = {           # (kernel kind, precision) -> bytes per launch
    ("dt", "fp64"): 79187186.3, ("dt", "mixed32"): 79187117.7,
    ("recon", "fp64"): 679224807.6, ("recon", "mixed32"): 632921917.0,   # with the boundary ghost pre-pass
    ("flux", "fp64"): 727239387.9, ("flux", "mixed32"): 500359022.7,
    ("cell", "fp64"): 563416994.5, ("cell", "mixed32"): 382768747.7,
    ("low_face", "fp64"): 183610947.0, ("low_face", "mixed32"): 175542777.9,
    ("low_cell", "fp64"): 256259519.0, ("low_cell", "mixed32"): 242142920.1,  # 1 forcing + 5 step launches
    ("sweep", "fp64"): 56983133.4, ("sweep", "mixed32"): 42802570.1,          # average over colour classes
    ("prolong", "fp64"): 149334136.4, ("prolong", "mixed32"): 144102496.0,
    ("dt", "mixed32_r64"): 79187140.6, ("recon", "mixed32_r64"): 647552089.4,
    ("flux", "mixed32_r64"): 560739536.3, ("cell", "mixed32_r64"): 401388582.6,
    ("low_face", "mixed32_r64"): 175442471.6, ("low_cell", "mixed32_r64"): 242221521.3,
    ("sweep", "mixed32_r64"): 42814922.6, ("prolong", "mixed32_r64"): 143886307.0,
}


def workload(name):
    import paper_2109_09965_amd.inputs as I
    if name == "sphere":
        mesh = I.sphere_case_mesh()
        Ma, Re = 0.25, 100.0
        Winf = I.free_stream(3, Ma)
        kw = dict(W_inf=Winf, mu=Ma * 1.0 / Re, Pr=0.72, area_ref=np.pi * 0.25)
        desc = ("3-D laminar sphere, hybrid O-grid on a cubed sphere 6x28x28 surface quads x 40 layers "
                "(20 hex, 10 prism, 10 tet), "
                "Ma 0.25, Re 100, Pr 0.72, adiabatic no-slip wall, S2O4 + 6 implicit steps x 2 sweeps")
    elif name == "cylinder":
        mesh = I.cylinder_case_mesh()
        Winf = I.free_stream(2, 0.2)
        kw = dict(W_inf=Winf, area_ref=1.0)
        desc = ("2-D inviscid cylinder, O-mesh 64x32 quads split into 4096 triangles, Ma 0.2, slip wall, "
                "S2O4 + 6 implicit steps x 2 sweeps")
    else:
        raise SystemExit(f"unknown workload {name}")
    return mesh, kw, desc


def kernels_sha256():
    import hashlib
    path = os.path.join(ROOT, "paper_2109_09965_amd", "csrc", "kernels.h")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def layout_sizes(d):
    nv = d + 2
    nk = 5 if d == 2 else 9
    nq = 3 if d == 2 else 6
    return dict(nv=nv, nk=nk, nq=nq, ns=4 if d == 2 else 8, nsym=nk * (nk + 1) // 2, sr=nv + d * nv,
                gr=d + nq + 1, er=d + 1 + nq + nv + nk * nv, fs=2 * nv + 2 * d * nv, fs_planar=4 * nv + d)


def sweep_sequence(n_colour, n_sweeps=2):
    """Colour classes visited by the sweeps of one implicit step (ascending,
    descending, repeated; a colour repeated back to back is visited once)."""
    seq = []
    for _ in range(n_sweeps):
        seq += list(range(n_colour)) + list(range(n_colour - 1, -1, -1))
    out = []
    for c in seq:
        if not out or out[-1] != c:
            out.append(c)
    return out


def algorithmic_bytes(mesh, lm, rbytes, sbytes=8):
    """Bytes per launch of each kernel kind, averaged over its launches in
    one S2O4 cycle: every distinct array element the kernel reads or writes
    by definition counted once per launch (no credit for cache re-reads, no
    charge for misses).  FP64 8 B, high-order arrays rbytes (8 FP64, 4
    mixed), low-level increments dU sbytes (8 FP64, 4 mixed), int32 4 B,
    int2 8 B.  Returns {kind: (bytes, launches)}."""
    d = mesh["dim"]
    z = layout_sizes(d)
    nv, ns, sr, gr, er, fs, nk = z["nv"], z["ns"], z["sr"], z["gr"], z["er"], z["fs"], z["nk"]
    NC, NF, NG, NB = lm.n_cell, lm.n_face, lm.n_gp, lm.info.n_boundary_face
    R = rbytes
    out = {}
    out["dt"] = (NC * (8 * nv + 8 + 4), 1)
    ghost = NB * (8 * sr + 4 + 4 + 4 + 8 * d + 8 + 8 * (nv + d * nv))
    recon = (NC * (8 * sr + 8 * gr + R * z["nsym"] + 8 * ns + R * er) + NB * (8 * nk + 8 * (nv + d * nv)))
    out["recon"] = (recon + ghost, 3)          # ghost pre-pass timed with the reconstruction
    face_idx = NF * (5 * 4 + 8 * d) + 4
    gp = NG * 8 * (2 * d + 1)
    # face records: F0, Ft, header and one Gauss-Green group for a planar face,
    # one group per axis otherwise
    NP = lm.info.n_planar_faces
    frec = R * (NP * z["fs_planar"] + (NF - NP) * fs)
    flux_grad = NC * R * er + gp + face_idx + frec
    flux_r1 = NC * R * er + gp + face_idx + NF * R * 2 * nv
    out["flux"] = ((2 * flux_grad + flux_r1) / 3.0, 3)
    cell_common = NC * (8 * ns + 4 + 8)
    st0 = cell_common + frec + NC * 8 * (nv + 3 * nv + sr + d * nv)
    st1 = cell_common + frec + NC * 8 * (3 * nv + d * nv + sr)
    r1 = cell_common + NF * R * 2 * nv + NC * 8 * nv
    out["cell"] = ((st0 + st1 + r1) / 3.0, 3)
    own, nb = mesh["face_owner"], mesh["face_neigh"]
    # indices, S, avec; lowf, S lam writes; the cells' volumes; each cell's
    # state once (a face reads both of its cells, every cell is read by all
    # its faces: counted once by definition)
    lf_common = NF * (4 * 3 + 8 + 8 * d) + 8 * NF * (nv + 1) + 8 * NC
    lf_force = lf_common + 8 * nv * NC                            # W
    lf_step = lf_common + (8 + sbytes) * nv * NC                  # U and dU
    out["low_face"] = ((lf_force + 5 * lf_step) / 6.0, 6)         # the first step reuses the forcing's
    lc_common = NC * (8 * ns + 4) + NF * 8 * (nv + 1)
    lc_force = lc_common + NC * (8 * (5 * nv + 2 + 1) + sbytes * nv)   # R1, W; Sf, U, RHS; vol, h; D; dU
    lc_step = lc_common + NC * (8 * (4 * nv + 2 + 1) + 2 * sbytes * nv)  # U, Sf; U, RHS; vol, h; D; dU r/w
    out["low_cell"] = ((lc_force + 5 * lc_step) / 6.0, 6)
    # sweeps, per colour class c: per cell of c its slots, case, RHS, D and
    # the dU write; the face record of every interior face of c (faces of an
    # independent set are distinct); the U, dU record of every distinct
    # neighbour
    colour = np.asarray(lm.colour)
    inner = nb >= 0
    a, b2 = own[inner], nb[inner]
    n_face_c = np.bincount(colour[a], minlength=lm.n_colour) + np.bincount(colour[b2], minlength=lm.n_colour)
    # distinct (colour of the cell, neighbour) pairs
    pairs = np.unique(np.concatenate([colour[a].astype(np.int64) * NC + b2, colour[b2].astype(np.int64) * NC + a]))
    n_nb_c = np.bincount(pairs // NC, minlength=lm.n_colour)
    n_cell_c = np.bincount(colour, minlength=lm.n_colour)
    by_colour = (n_cell_c * (8 * ns + 4 + 8 * nv + 8 + sbytes * nv) + n_face_c * 8 * (d + 1)
                 + n_nb_c * (8 + sbytes) * nv)
    seq = sweep_sequence(lm.n_colour)
    out["sweep"] = (float(sum(by_colour[c] for c in seq)) / len(seq), 6 * len(seq))
    out["prolong"] = (NC * (8 * (nv + 2 * nv + 1) + sbytes * nv), 1)
    return out


def converge_report(mesh, lm, kw, drop=1e-10, max_cycles=3000):
    """The workload run to a residual drop from the uniform start: FP64, and
    MIXED32_R64 until it levels off at its FP32 floor, then finished in
    FP64 to the same drop.  Reports cycles, seconds, drag coefficient and
    the mixed state's error against the FP64 converged state (L2 and max,
    relative), before and after the FP64 finish."""
    import torch
    import paper_2109_09965_amd as cg
    import paper_2109_09965_amd.inputs as I
    W0, dW0 = I.uniform_state(mesh, kw["W_inf"])

    def solve(b, tol, tol_abs, cycles):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep, hist = b.solve(max_cycles=cycles, tol=tol, tol_abs=tol_abs, check_every=8, history=True)
        torch.cuda.synchronize()
        return rep[0], hist[0][:rep[0]["cycles"]], time.perf_counter() - t0

    b = cg.Batch([lm], [cg.Params(**kw)])
    b.upload(0, W0, dW0)
    b.autotune()
    r64, h64, t64 = solve(b, drop, False, max_cycles)
    W64, _ = b.download(0)
    cd64 = r64["cd"]
    del b
    out = dict(fp64=dict(cycles=r64["cycles"], seconds=t64, res_drop=float(h64[-1] / h64[0]), converged=r64["converged"],
                         cd=cd64))
    # mixed: run until Res stops improving by 1 % over 100 cycles (its floor)
    bm = cg.Batch([lm], [cg.Params(**kw)], precision=cg.MIXED32_R64)
    bm.upload(0, W0, dW0)
    bm.autotune()
    tm, hm, cyc = 0.0, [], 0
    best, best_at = np.inf, 0
    while cyc < max_cycles:
        rm, h, t = solve(bm, drop, False, 50)
        tm += t
        hm += list(h)
        cyc += rm["cycles"]
        for k, r in enumerate(h):
            if r < 0.99 * best:
                best, best_at = r, cyc - len(h) + k + 1
        if rm["converged"] or cyc - best_at >= 100:
            break
    Wm, dWm = bm.download(0)
    cdm = rm["cd"]
    del bm
    err = lambda A: (float(np.linalg.norm(A - W64) / np.linalg.norm(W64)), float(np.abs(A - W64).max() / np.abs(W64).max()))
    e_floor = err(Wm)
    bf = cg.Batch([lm], [cg.Params(**kw)])
    bf.upload(0, Wm, dWm)
    bf.autotune()
    rf, hf, tf = solve(bf, drop * hm[0], True, max_cycles)
    Wf, _ = bf.download(0)
    del bf
    out["mixed32_r64"] = dict(cycles_mixed=cyc, cycles_fp64_finish=rf["cycles"], seconds=tm + tf,
                              floor_drop=float(min(hm) / hm[0]), cd_at_floor=cdm,
                              cd=rf["cd"], converged=rf["converged"],
                              l2_rel_err_at_floor=e_floor[0], max_rel_err_at_floor=e_floor[1],
                              l2_rel_err=err(Wf)[0], max_rel_err=err(Wf)[1])
    return out


def cpu_baseline(mesh, kw):
    """The oracle as it stands (plain FP64 C, one host thread) timed on one
    whole cycle of the benchmark mesh from the same uniform start."""
    import oracle
    import paper_2109_09965_amd.inputs as I
    t0 = time.perf_counter()
    om = oracle.Mesh(mesh)
    t_prep = time.perf_counter() - t0
    s = oracle.Solver(om, oracle.Params(**{k: v for k, v in kw.items() if k != "area_ref"}))
    W, dW = I.uniform_state(mesh, kw["W_inf"])
    t0 = time.perf_counter()
    s.cycle(W, dW)
    t = time.perf_counter() - t0
    return dict(value=mesh["n_cell"] / t, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"1 cycle of the benchmark mesh ({mesh['n_cell']} cells), FP64, 1 thread, {t:.1f} s "
                       f"(oracle geometry and colouring {t_prep:.1f} s, not timed)")


def run_batch(args):
    """64 seeded cylinder cases of uneven size stepped together (one launch
    per kernel covers every case), FP64 and MIXED32, as captured graphs of G
    cycles; then the same cases one at a time in FP64, each with its own
    graph.  value = batched FP64 cell-updates/s."""
    import torch
    import paper_2109_09965_amd as cg
    import paper_2109_09965_amd.inputs as I
    cases = I.batch_cases(64, 2109)
    meshes = [I.batch_case_mesh(c) for c in cases]
    winf = [I.free_stream(2, c["mach"], c["aoa"]) for c in cases]
    lms = [cg.Mesh(m) for m in meshes]
    # transonic cases (Ma > 0.4) with the full gas-kinetic solution and
    # nonlinear weights, as the paper runs its transonic flows
    params = [cg.Params(W_inf=w, flux_kind=cg.FLUX_FULL if c["transonic"] else cg.FLUX_SMOOTH,
                        weno_eps=args.weno_eps if c["transonic"] else 0.0) for c, w in zip(cases, winf)]
    NC = sum(lm.n_cell for lm in lms)
    G = max(g for g in (1, 2, 4, 5) if args.steps % g == 0)

    def run(idx, prec):
        b = cg.Batch([lms[i] for i in idx], [params[i] for i in idx], precision=prec)
        for k, i in enumerate(idx):
            W, dW = I.uniform_state(meshes[i], winf[i])
            b.upload(k, W, dW)
        if not args.no_autotune:
            b.autotune()
        for _ in range(args.warmup):
            b.cycle()
        b.graph_create(G)
        hist = torch.zeros(G * len(idx), dtype=torch.float64, device="cuda")
        b.graph_launch(hist)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps // G):
            b.graph_launch(hist)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res = hist.cpu().numpy().reshape(G, len(idx))
        del b
        return t, int(np.isfinite(res[-1]).sum())

    out = {}
    for name, prec in (("fp64", cg.FP64), ("mixed32", cg.MIXED32)):
        t, ok = run(list(range(len(cases))), prec)
        out[name] = (NC * args.steps / t, ok)
    t_one, ok_one = 0.0, 0
    for i in range(len(cases)):
        t, ok = run([i], cg.FP64)
        t_one += t
        ok_one += ok
    one = NC * args.steps / t_one
    sizes = sorted({lm.n_cell for lm in lms})
    line = dict(metric="cell-updates/s per p-MG cycle", value=out["fp64"][0], unit="cell-updates/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=1e3 * NC / out["fp64"][0],
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
                data="synthetic (seeded cylinder meshes and free streams, uniform start)",
                config=dict(workload="batch of 64 inviscid cylinders (n_theta in {32,64,128,256}, n_r = n_theta/2, "
                            "Ma ~ U[0.1,0.6], AoA ~ U[-5,5] deg; Ma > 0.4 with the full gas-kinetic solution "
                            f"and nonlinear weights, eps {args.weno_eps:g}), one launch per kernel for all cases, "
                            f"graphs of {G} cycles", cases=len(cases), cells=NC, case_sizes=sizes,
                            transonic_cases=sum(c["transonic"] for c in cases)),
                mixed32_value=out["mixed32"][0], one_at_a_time_fp64_value=one,
                batched_speedup_fp64=out["fp64"][0] / one, batched_speedup_mixed32=out["mixed32"][0] / one,
                cases_finite_after_all_steps=dict(fp64=out["fp64"][1], mixed32=out["mixed32"][1],
                                                  one_at_a_time=ok_one))
    print(json.dumps(line), flush=True)


def _serve_mesh(spec):
    import paper_2109_09965_amd.inputs as I
    return I.serve_mesh(spec)


def run_serve(args):
    """Serving trace: seeded Poisson arrivals (20 requests/s) of steady-solve
    requests, 70 % viscous cylinders and 30 % hybrid spheres, served by the
    continuous-batching server (pools admitted by HBM footprint) and, for
    comparison, strictly one case at a time in FP64 in arrival order.
    value = the server's aggregate cell-updates/s."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import paper_2109_09965_amd.inputs as I
    trace = I.serve_trace(args.requests, seed=9965, rate=20.0)
    # the client prepares its meshes before the trace starts (worker
    # processes forked before anything touches the GPU)
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1), mp_context=mp.get_context("fork")) as ex:
        meshes = list(ex.map(_serve_mesh, trace, chunksize=1))
    import paper_2109_09965_amd as cg
    from paper_2109_09965_amd.serve import Request, Server, summarize
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        lms = list(ex.map(cg.Mesh, meshes))
    import torch
    prec = {"fp64": cg.FP64, "mixed32": cg.MIXED32, "mixed32_r64": cg.MIXED32_R64}[args.precision]
    tol = 1e-10 if prec == cg.FP64 else 1e-8

    def requests():
        out = []
        for k, (spec, m, lm) in enumerate(zip(trace, meshes, lms)):
            w = I.free_stream(spec["dim"], spec["mach"], spec["aoa"])
            W, dW = I.uniform_state(m, w)
            # transonic requests (Ma > 0.4) with the full gas-kinetic solution and nonlinear weights
            tr = spec["mach"] > 0.4
            p = cg.Params(W_inf=w, mu=spec["mach"] / spec["re"], Pr=0.72,
                          flux_kind=cg.FLUX_FULL if tr else cg.FLUX_SMOOTH, weno_eps=1e-2 if tr else 0.0)
            out.append(Request(rid=k, arrival=spec["arrival"], mesh=lm, params=p, W0=W, dW0=dW, tol=tol))
        return out

    free = torch.cuda.mem_get_info()[0]
    budget = args.budget_gb * 1e9 if args.budget_gb else 0.9 * free
    srv = Server(budget, precision=prec, max_cases=64, epoch_cycles=8, max_cycles=4000, stall_cycles=400,
                 max_resident={2: args.resident_2d, 3: args.resident_3d}, finish_fp64=not args.no_fp64_finish)
    reqs = requests()

    def progress(r):
        print(f"served {r.rid}: dim {r.mesh.dim} cells {r.mesh.n_cell} {r.status} after {r.cycles} cycles "
              f"({r.cycles_fp64} in FP64), "
              f"time-to-steady {r.done - r.arrival:.2f} s", file=sys.stderr, flush=True)

    served = srv.run(reqs, log=progress)
    del srv
    torch.cuda.empty_cache()
    # one case at a time, FP64, arrival order, the same tolerance rule
    base = None
    if not args.no_sequential:
        seq = requests()
        t0 = time.perf_counter()
        work = 0
        for r in seq:
            while time.perf_counter() - t0 < r.arrival:
                time.sleep(0.001)
            b = cg.Batch([r.mesh], [r.params])
            r.admitted = time.perf_counter() - t0
            b.upload(0, r.W0, r.dW0)
            rep, hist = b.solve(max_cycles=4000, tol=r.tol, tol_abs=True, check_every=8, history=True)
            r.cycles = rep[0]["cycles"]
            r.W, _ = b.download(0)
            r.done = time.perf_counter() - t0
            r.status = "converged" if rep[0]["converged"] else "not_converged"
            work += r.mesh.n_cell * r.cycles
            del b
            print(f"one at a time {r.rid}: {r.status} after {r.cycles} cycles, time-to-steady "
                  f"{r.done - r.arrival:.2f} s", file=sys.stderr, flush=True)
        base = summarize(seq, work, time.perf_counter() - t0)
    n2 = sum(1 for t in trace if t["dim"] == 2)
    line = dict(metric="aggregate cell-updates/s and p50/p99 time-to-steady (serving)", value=served["cell_updates_per_s"],
                unit="cell-updates/s", n_gpus=1, steps=len(trace), warmup=0, ms_per_step=None,
                higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f64" if prec == cg.FP64 else "f32+f64", data="synthetic (seeded request trace and meshes)",
                config=dict(workload=f"serving trace: {len(trace)} requests at 20/s ({n2} viscous cylinders "
                                     f"n_theta 32..256, {len(trace) - n2} hybrid cubed spheres; Ma ~ U[0.1,0.5], "
                                     f"Re ~ U[50,300]), tol Res <= {tol:g}, at most 4000 cycles",
                            precision=args.precision.upper(), budget_gb=budget / 1e9,
                            resident_cells={"2d": args.resident_2d, "3d": args.resident_3d}),
                served=served, one_at_a_time_fp64=base)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sphere", choices=["sphere", "cylinder", "batch64", "serve"])
    ap.add_argument("--requests", type=int, default=256, help="serving trace length")
    ap.add_argument("--budget-gb", type=float, default=0.0, help="serving HBM budget (default 0.9 x free)")
    ap.add_argument("--no-sequential", action="store_true", help="serving: skip the one-at-a-time baseline")
    ap.add_argument("--no-fp64-finish", action="store_true",
                    help="serving, mixed precisions: do not finish cases at the FP32 floor in FP64")
    ap.add_argument("--resident-2d", type=int, default=200_000, help="serving: cells a 2-D pool runs at once")
    ap.add_argument("--resident-3d", type=int, default=500_000, help="serving: cells a 3-D pool runs at once")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed32", "mixed32_r64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="FP64 only: skip the MIXED32 and MIXED32_R64 legs")
    ap.add_argument("--weno-eps", type=float, default=1e-2, help="batch64: epsilon of the transonic cases' weights")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--no-converge", action="store_true", help="skip the run to a 1e-10 residual drop")
    ap.add_argument("--order-tile", type=int, default=0,
                    help="cells per tile of the library cell order (0 = library default)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (counter calibration)")
    ap.add_argument("--gather-calib", type=int, default=0, metavar="MIB",
                    help="only run 5 gathers of MIB MiB in whole 128-byte rows, random row order (counter calibration)")
    args = ap.parse_args()
    if args.gather_calib:
        # every 128-byte row of the source read once, in a seeded random
        # order, plus the 8-byte row indices; the output written in order
        import torch
        rows = args.gather_calib * (1 << 20) // 128
        g = torch.Generator(device="cpu").manual_seed(2109)
        perm = torch.randperm(rows, generator=g).cuda()
        src = torch.ones(rows, 16, dtype=torch.float64, device="cuda")
        out = torch.empty_like(src)
        for _ in range(5):
            torch.index_select(src, 0, perm, out=out)
        torch.cuda.synchronize()
        print(json.dumps(dict(gather_bytes_each=rows * 128, index_bytes_each=rows * 8, gathers=5)))
        return
    if args.copy_calib:
        import torch
        n = args.copy_calib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes_each=n * 8, copies=5)))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent cases shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        run_batch(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return

    import torch
    import paper_2109_09965_amd as cg
    import paper_2109_09965_amd.inputs as I

    mesh, kw, desc = workload(args.workload)
    lm = cg.Mesh(mesh, order_tile=args.order_tile)
    main_prec = args.precision
    out = measure(mesh, lm, kw, main_prec, args)
    value = out.pop("value")
    line = dict(metric="cell-updates/s per p-MG cycle", value=value, unit="cell-updates/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=out.pop("ms_per_step"),
                higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f64" if main_prec == "fp64" else "f32+f64",
                data="synthetic (seeded mesh generator, uniform free-stream start)",
                config=dict(workload=desc, cells=lm.n_cell, faces=lm.n_face, gauss_points=lm.n_gp,
                            colours=lm.n_colour, precision=main_prec.upper(), time_scheme="S2O4", implicit_steps=6,
                            sweeps=2, launch_shapes=out.pop("launch_shapes"),
                            order_tile=args.order_tile or cg.ORDER_TILE_DEFAULT))
    line["roofline"] = out.pop("roofline")
    line.update(out)
    if main_prec == "fp64" and not args.no_mixed:
        # the FP32 half of the metric on the same mesh, same launch procedure
        for name in ("mixed32", "mixed32_r64"):
            o = measure(mesh, lm, kw, name, args)
            line[name] = dict(value=o["value"], unit="cell-updates/s", ms_per_step=o["ms_per_step"], dtype="f32+f64",
                              roofline=o["roofline"], kernels=o["kernels"])
    if args.workload == "sphere" and not args.no_converge:
        line["convergence"] = converge_report(mesh, lm, kw)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(mesh, kw)
    print(json.dumps(line), flush=True)


def measure(mesh, lm, kw, prec_name, args):
    """Tune the launch shapes, run the warm-up cycles, time args.steps cycles
    with HIP-event kernel timing on the launch stream, then time them again
    without events, eagerly and as captured graphs; value from the faster of
    the last two.  Returns the value, the kernel breakdown and the dominant
    kernel's roofline."""
    import torch
    import paper_2109_09965_amd as cg
    import paper_2109_09965_amd.inputs as I
    prec = {"fp64": cg.FP64, "mixed32": cg.MIXED32, "mixed32_r64": cg.MIXED32_R64}[prec_name]
    b = cg.Batch([lm], [cg.Params(**kw)], precision=prec)
    W, dW = I.uniform_state(mesh, kw["W_inf"])
    b.upload(0, W, dW)
    picks = None if args.no_autotune else b.autotune()     # launch shapes, before the timed region
    res = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        b.cycle(res)
    torch.cuda.synchronize()
    b.timing(True)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        b.cycle(res)
    torch.cuda.synchronize()
    kt = b.timing_read()
    b.timing(False)
    # the timed region above carries event records; time once more without
    # them, eagerly and as one captured graph of all the steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.cycle(res)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    # blocks of G cycles captured once and replayed (very large graphs replay slowly)
    G = max(g for g in (1, 2, 4, 5) if args.steps % g == 0)
    b.graph_create(G)
    hist = torch.zeros(G, dtype=torch.float64, device="cuda")
    b.graph_launch(hist)      # warm replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps // G):
        b.graph_launch(hist)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    res_graph = float(hist.cpu()[-1])
    t_clean = min(t_eager, t_graph)
    NC, NG = lm.n_cell, lm.n_gp
    value = NC * args.steps / t_clean
    # dominant kernel by total time; every kernel's achieved bandwidth
    dom = max(kt, key=lambda k: kt[k][0])
    tot_ms = sum(v[0] for v in kt.values())
    model = algorithmic_bytes(mesh, lm, 8 if prec == cg.FP64 else 4, 8 if prec == cg.FP64 else 4)
    per_kernel_gbs = {}
    for k, (ms, n) in kt.items():
        if n and k in model:
            per_kernel_gbs[k] = model[k][0] / (ms / n * 1e-3) / 1e9
    avg_ms = kt[dom][0] / kt[dom][1]
    traffic = PROFILED_TRAFFIC.get((dom, prec_name)) if kernels_sha256() == PROFILED_KERNELS_SHA256 else None
    if dom == "flux":
        flop = FLUX_FLOP_PER_GP[prec_name] * NG
        ach = flop / (avg_ms * 1e-3) / 1e12
        peak = VALU_PEAK_TFLOPS[prec_name]
        rf = dict(bound="alu", kernel=dom, achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                  traffic=traffic, flop_per_launch=flop, alg_bytes_per_launch=model[dom][0], avg_launch_ms=avg_ms)
        if prec_name != "fp64":
            rf["peak_packed_fp32"] = FP32_PACKED_PEAK_TFLOPS
    else:
        byt = model[dom][0]
        ach = byt / (avg_ms * 1e-3) / 1e9
        rf = dict(bound="hbm", kernel=dom, achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                  traffic=traffic, bytes_per_launch=byt, avg_launch_ms=avg_ms)
    breakdown = {k: dict(ms_per_step=v[0] / args.steps, launches_per_step=v[1] / args.steps,
                         share=v[0] / tot_ms if tot_ms else 0.0, alg_gbs=per_kernel_gbs.get(k))
                 for k, v in kt.items()}
    del b
    return dict(value=value, ms_per_step=1e3 * t_clean / args.steps, launch_shapes=picks, roofline=rf,
                kernels=breakdown, res_last=float(res.cpu()[0]), res_after_graph=res_graph,
                eager_ms_per_step=1e3 * t_eager / args.steps, graph_ms_per_step=1e3 * t_graph / args.steps)


if __name__ == "__main__":
    main()
