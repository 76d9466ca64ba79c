"""Converged-state parity: the HIP path run to its steady state from the
uniform free stream against the oracle's steady state on the same inputs
(tests/golden/converged_*.npz, written by make_converged_states.py, which
runs the oracle alone).  The steady state is the fixed point of the
two-level cycle (Sec. 3): the FP64 path must reach it within 1e-9 of each
variable's scale, in the same number of cycles to a 1e-10 residual drop
(within one cycle at the threshold).  The mixed-precision paths are held to
their stated bounds against the same oracle state."""
import os

import numpy as np
import pytest

import paper_2109_09965_amd as cg
import paper_2109_09965_amd.inputs as I

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# the same cases as tests/golden/make_converged_states.py
CASES = {
    "cylinder_re40": dict(mesh=lambda: I.cylinder_mesh(32, 16, wall=I.BC_NOSLIP_ADIABATIC), dim=2, mach=0.15,
                          re=40.0),
    "sphere_re20": dict(mesh=lambda: I.cubed_sphere_mesh(3, 8, 4, 2, wall=I.BC_NOSLIP_ADIABATIC), dim=3,
                        mach=0.25, re=20.0),
}
# stated bounds of the mixed paths' steady states against the FP64 oracle's
# (relative to each variable's scale): their FP32 explicit stages leave a
# residual floor near a 1e-5 drop, so the state stops there.  Measured on
# MI355X: MIXED32 1.3e-5 (cylinder) and 2.1e-5 (sphere), MIXED32_R64 2.0e-6
# and 5.5e-5 (the sphere's cross-flow momentum, whose scale is small)
MIXED_BOUND = {cg.MIXED32: 1e-4, cg.MIXED32_R64: 1e-4}


def run_gpu(name, precision, n_cycles):
    import torch
    case = CASES[name]
    mesh = case["mesh"]()
    Winf = I.free_stream(case["dim"], case["mach"])
    b = cg.Batch([cg.Mesh(mesh)], [cg.Params(W_inf=Winf, mu=case["mach"] / case["re"], Pr=0.72)],
                 precision=precision)
    W0, dW0 = I.uniform_state(mesh, Winf)
    b.upload(0, W0, dW0)
    blk = 8
    b.graph_create(blk)
    hist = torch.zeros(blk, dtype=torch.float64, device="cuda")
    res = []
    for _ in range(n_cycles // blk):
        b.graph_launch(hist)
        res.extend(hist.cpu().numpy().tolist())
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(n_cycles % blk):
        b.cycle(one)
        res.append(float(one.cpu()[0]))
    W, dW = b.download(0)
    return W, dW, np.array(res)


def first_below(res, drop):
    k = np.flatnonzero(res <= drop * res[0])
    return int(k[0]) if len(k) else None


def rel_err(A, B):
    """max over elements of |A - B| / (scale of the variable), scale = max |B_v|"""
    axis = tuple(range(A.ndim - 1))
    if A.ndim == 2:
        scale = np.abs(B).max(1, keepdims=True)
    else:
        scale = np.abs(B).max(axis=(0, 2), keepdims=True)
    return float((np.abs(A - B) / scale).max())


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(CASES))
def test_fp64_converged_state_matches_oracle(name):
    fx = np.load(os.path.join(GOLDEN, f"converged_{name}.npz"))
    n = int(fx["cycles"])
    print(f"converged parity {name}: {n} cycles (FP64)", flush=True)
    W, dW, res = run_gpu(name, cg.FP64, n)
    eW, edW = rel_err(W, fx["W"]), rel_err(dW, fx["dW"])
    print(f"{name}: FP64 state vs oracle {eW:.2e} (W), {edW:.2e} (grad W); Res drop {res[-1] / res[0]:.2e}",
          flush=True)
    assert eW <= 1e-9 and edW <= 1e-9, (eW, edW)
    ko, kg = first_below(fx["res"], 1e-10), first_below(res, 1e-10)
    assert ko is not None and kg is not None and abs(ko - kg) <= 1, (ko, kg)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [cg.MIXED32, cg.MIXED32_R64])
@pytest.mark.parametrize("name", list(CASES))
def test_mixed_converged_state_within_its_bound(name, precision):
    fx = np.load(os.path.join(GOLDEN, f"converged_{name}.npz"))
    n = int(fx["cycles"])
    W, dW, res = run_gpu(name, precision, n)
    eW, edW = rel_err(W, fx["W"]), rel_err(dW, fx["dW"])
    print(f"{name}: precision {precision} state vs FP64 oracle {eW:.2e} (W), {edW:.2e} (grad W); "
          f"Res drop floor {res.min() / res[0]:.2e}", flush=True)
    assert eW <= MIXED_BOUND[precision], eW
