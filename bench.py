"""Benchmark: cell-updates/s of the p-multigrid CGKS cycle on one MI355X.

One step = one two-level cycle (S2O4 high-order step with Gauss-Green
gradient update, high-order residual, KFVS forcing, 6 implicit steps of 2
multicolour point-relaxation sweeps, prolongation, Res) on every cell of the
workload.  Default workload: 3-D hybrid sphere O-grid on a cubed-sphere
surface (6 x 28 x 28 quads, 40 layers: 20 hex, 10 prism, 10 tet; 470,400
cells), Ma 0.25, Re 100, Pr 0.72, no-slip isothermal wall, FP64.  Inputs are resident on the device
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
FP64_VECTOR_TFLOPS = 78.6      # MI355X FP64 vector


def workload(name):
    import paper_2109_09965_amd.inputs as I
    if name == "sphere":
        mesh = I.sphere_case_mesh()
        Ma, Re = 0.25, 100.0
        Winf = I.free_stream(3, Ma)
        kw = dict(W_inf=Winf, mu=Ma * 1.0 / Re, Pr=0.72, T_wall=1.0 / 1.4)
        desc = ("3-D laminar sphere, hybrid O-grid on a cubed sphere 6x28x28 surface quads x 40 layers "
                "(20 hex, 10 prism, 10 tet), "
                "Ma 0.25, Re 100, Pr 0.72, isothermal no-slip wall, S2O4 + 6 implicit steps x 2 sweeps")
    elif name == "cylinder":
        mesh = I.cylinder_case_mesh()
        Winf = I.free_stream(2, 0.2)
        kw = dict(W_inf=Winf)
        desc = ("2-D inviscid cylinder, O-mesh 64x32 quads split into 4096 triangles, Ma 0.2, slip wall, "
                "S2O4 + 6 implicit steps x 2 sweeps")
    else:
        raise SystemExit(f"unknown workload {name}")
    return mesh, kw, desc


def algorithmic_bytes(kind, d, NC, NF, NG, NB):
    """Distinct array elements each kernel reads or writes per launch (FP64
    values 8 B, int32 indices 4 B), no credit for cache reuse."""
    nv = d + 2
    nk = 5 if d == 2 else 9
    nq = 3 if d == 2 else 6
    ns = 4 if d == 2 else 8
    nsym = nk * (nk + 1) // 2
    if kind == "flux":
        return (NG * (8 * (2 * d + 1 + 4 * nv) + 4) + NF * (4 * 4 + 8 * d)
                + NC * 8 * (nv + nk * nv + d + 1 + nq))
    if kind == "recon":
        return (NC * (8 * (nv + d * nv + d + 1 + nq + nsym + nk * nv) + 4 * (2 * ns + 1))
                + NF * 8 * d + NB * (8 * (nk + d + 1) + 8))
    if kind == "cell":  # stage-0 variant
        return (NC * (4 * (ns + 1) + 8 * (1 + 5 * nv + 2 * d * nv)) + NG * 8 * (4 * nv + d) + NF * 4)
    raise KeyError(kind)


def cpu_baseline(seconds_hint=30.0):
    """The oracle as it stands, on a reduced hybrid sphere built the same way
    (cubed sphere 6 x 14 x 14 surface quads x 20 layers), single thread."""
    import oracle
    import paper_2109_09965_amd.inputs as I
    mesh = I.cubed_sphere_mesh(14, 20, 10, 5, r_far=15.0, ratio=1.08)
    Ma, Re = 0.25, 100.0
    Winf = I.free_stream(3, Ma)
    s = oracle.Solver(oracle.Mesh(mesh), oracle.Params(W_inf=Winf, mu=Ma / Re, Pr=0.72, T_wall=1 / 1.4))
    W, dW = I.uniform_state(mesh, Winf)
    n = 0
    t0 = time.perf_counter()
    while True:
        s.cycle(W, dW)
        n += 1
        if time.perf_counter() - t0 > seconds_hint / 3 or n >= 3:
            break
    t = time.perf_counter() - t0
    return dict(value=mesh["n_cell"] * n / t, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"{n} cycle(s) of the 6x14x14x20 cubed-sphere hybrid sphere ({mesh['n_cell']} cells), FP64, "
                       f"1 thread, {t:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sphere", choices=["sphere", "cylinder"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (counter calibration)")
    args = ap.parse_args()
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
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent cases shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2109_09965_amd as cg
    import paper_2109_09965_amd.inputs as I

    mesh, kw, desc = workload(args.workload)
    lm = cg.Mesh(mesh)
    prec = cg.MIXED32 if args.precision == "mixed32" else cg.FP64
    b = cg.Batch([lm], [cg.Params(**kw)], precision=prec)
    W, dW = I.uniform_state(mesh, kw["W_inf"])
    b.upload(0, W, dW)
    res = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        b.cycle(res)
    torch.cuda.synchronize()
    b.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.cycle(res)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
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
    NC, NF, NG, NB = lm.n_cell, lm.n_face, lm.n_gp, lm.info.n_boundary_face
    d = mesh["dim"]
    value = NC * args.steps / t_clean
    # dominant kernel by total time
    dom = max(kt, key=lambda k: kt[k][0])
    tot_ms = sum(v[0] for v in kt.values())
    rf = None
    if dom in ("flux", "recon", "cell"):
        avg_ms = kt[dom][0] / kt[dom][1]
        byt = algorithmic_bytes(dom, d, NC, NF, NG, NB)
        ach = byt / (avg_ms * 1e-3) / 1e9
        rf = dict(bound="hbm", kernel=dom, achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                  traffic=None, bytes_per_launch=byt, avg_launch_ms=avg_ms)
    breakdown = {k: dict(ms_per_step=v[0] / args.steps, launches_per_step=v[1] / args.steps,
                         share=v[0] / tot_ms if tot_ms else 0.0) for k, v in kt.items()}
    out = dict(metric="cell-updates/s per p-MG cycle", value=value, unit="cell-updates/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=1e3 * t_clean / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64" if prec == cg.FP64 else "f32+f64",
               data="synthetic (seeded mesh generator, uniform free-stream start)",
               config=dict(workload=desc, cells=NC, faces=NF, gauss_points=NG, colours=lm.n_colour,
                           precision=args.precision.upper(), time_scheme="S2O4", implicit_steps=6, sweeps=2),
               roofline=rf, kernels=breakdown, res_last=float(res.cpu()[0]), res_after_graph=res_graph,
               eager_ms_per_step=1e3 * t_eager / args.steps, graph_ms_per_step=1e3 * t_graph / args.steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
