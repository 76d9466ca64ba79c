"""Mixed-precision batches against the FP64 oracle and the FP64 GPU path.
MIXED32: FP32 reconstruction, interface states, gas-kinetic flux, face sums
and relaxation sweeps; FP64 cell averages, gradients, stage accumulation,
R1 accumulation, low-level state, KFVS flux and right-hand side, norms.
MIXED32_R64: the same with the residual pass R1 in FP64.

Stated bounds: after three cycles from a smooth perturbed state the cell
averages agree with the FP64 oracle to 2e-6 relative (max norm); on the
steady viscous cylinder the mixed paths level off at a residual drop below
1e-4 (the FP32 noise floor; MIXED32_R64 at or below MIXED32's) with cell
averages within 1e-5 relative of the converged FP64 state."""
import numpy as np
import pytest

import oracle
import paper_2109_09965_amd as cg
import paper_2109_09965_amd.inputs as I
from test_gpu_parity import make_case

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [cg.MIXED32, cg.MIXED32_R64])
@pytest.mark.parametrize("name", ["cyl2d_visc", "box2d_per", "box3d_per", "sphere", "cubed_sphere"])
def test_mixed_cycles_close_to_oracle(name, prec):
    m, kw, W, dW = make_case(name)
    b = cg.Batch([cg.Mesh(m)], [cg.Params(**kw)], precision=prec)
    b.upload(0, W, dW)
    s = oracle.Solver(oracle.Mesh(m), oracle.Params(**kw))
    W, dW = W.copy(), dW.copy()
    for k in range(3):
        s.cycle(W, dW)
        b.cycle()
        Wg, dWg = b.download(0)
        err = np.abs(Wg - W).max() / np.abs(W).max()
        gerr = np.abs(dWg - dW).max() / np.abs(dW).max()
        print(f"{name} precision {prec} cycle{k}: W rel err {err:.2e}, dW rel err {gerr:.2e}", flush=True)
    assert err <= 2e-6, err


def test_mixed_converges_to_fp64_state():
    m = I.cylinder_mesh(32, 16, wall=I.BC_NOSLIP_ISOTHERMAL)
    Winf = I.free_stream(2, 0.15)
    kw = dict(W_inf=Winf, mu=0.15 / 40, Pr=0.72)
    W, dW = I.uniform_state(m, Winf)
    out = {}
    for prec in (cg.FP64, cg.MIXED32, cg.MIXED32_R64):
        b = cg.Batch([cg.Mesh(m)], [cg.Params(**kw)], precision=prec)
        b.upload(0, W, dW)
        rep, hist = b.solve(max_cycles=1000, tol=1e-13, check_every=8, history=True)
        out[prec] = (b.download(0)[0], hist[0])
    W64, h64 = out[cg.FP64]
    assert h64[-1] / h64[0] < 1e-8
    floor = {}
    for prec in (cg.MIXED32, cg.MIXED32_R64):
        W32, h32 = out[prec]
        err = np.abs(W32 - W64).max() / np.abs(W64).max()
        floor[prec] = np.median(h32[-100:]) / h32[0]
        print(f"precision {prec}: converged-state rel err vs fp64 {err:.2e}; Res drop fp64 {h64[-1] / h64[0]:.2e}, "
              f"mixed floor {floor[prec]:.2e}", flush=True)
        assert h32.min() / h32[0] < 1e-4
        assert err <= 1e-5
    assert floor[cg.MIXED32_R64] <= 1.5 * floor[cg.MIXED32]
