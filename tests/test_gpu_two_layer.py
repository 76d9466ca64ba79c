"""The paper's practice of running 2-D cases on two-layer 3-D meshes
(Sec. 4, opening paragraph) against the library's native 2-D path, on the
GPU: the Re 40 cylinder (64 x 32 ring, no-slip adiabatic wall, Ma 0.15)
converged both ways.  The two discretisations differ by the cell-size
scaling of the reconstruction's gradient rows (h of a triangle against h
of its prism), so the states agree to the discretisation error, not to
round-off: drag within 0.5 % (measured 0.17 %: Cd 1.5210 native, 1.5184 on
two layers), cell averages within 3e-2 of each variable's scale (measured
1.7e-2, largest in the cross-flow momentum, whose scale is small).
The 3-D run must end z-uniform: no z momentum and both layers alike (the
multicolour sweeps update one layer before the other, so the layers differ
while the correction is nonzero and meet at the fixed point)."""
import numpy as np
import pytest

import paper_2109_09965_amd as cg
import paper_2109_09965_amd.inputs as I

pytestmark = pytest.mark.gpu


def solve(m, d, max_cycles=6000):
    Ma, Re = 0.15, 40.0
    w = I.free_stream(d, Ma)
    area = 1.0 if d == 2 else m["dz"] * 2      # unit span: the two layers' depth
    b = cg.Batch([cg.Mesh(m)], [cg.Params(W_inf=w, mu=Ma / Re, Pr=0.72, area_ref=area)])
    W, dW = I.uniform_state(m, w)
    b.upload(0, W, dW)
    rep, _ = b.solve(max_cycles=max_cycles, tol=1e-9, check_every=8)
    print(f"dim {d}: {rep[0]['cycles']} cycles, converged {rep[0]['converged']}, Cd {rep[0]['cd']:.5f}", flush=True)
    assert rep[0]["converged"], rep[0]
    return rep[0], b.download(0)[0]


def test_two_layer_cylinder_matches_native_2d():
    m2 = I.cylinder_mesh(64, 32, 0.5, ratio=1.1, first_spacing=0.09695, wall=I.BC_NOSLIP_ADIABATIC)
    m3 = I.extrude_two_layers(m2)
    r2, W2 = solve(m2, 2)
    r3, W3 = solve(m3, 3)
    n = m2["n_cell"]
    assert abs(r3["cd"] - r2["cd"]) <= 5e-3 * abs(r2["cd"])
    for l in range(2):
        Wl = W3[[0, 1, 2, 4], l * n:(l + 1) * n]
        err = (np.abs(Wl - W2).max(axis=1) / np.abs(W2).max(axis=1)).max()
        print(f"layer {l}: max difference from 2-D {err:.2e} of the variables' scales", flush=True)
        assert err <= 3e-2
    dz_mom = np.abs(W3[3]).max() / np.abs(W3[1]).max()
    layers = np.abs(W3[:, :n] - W3[:, n:]).max() / np.abs(W3).max()
    print(f"z momentum {dz_mom:.2e}, layer difference {layers:.2e}", flush=True)
    assert dz_mom <= 1e-10 and layers <= 1e-6          # measured 9.9e-14 and 1.5e-7 at the 1e-9 drop
