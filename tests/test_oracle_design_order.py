"""Design order of the oracle's high-order level on 3-D cells (Sec. 4's
compact quadratic reconstruction with the S2O4 and S1O2 time marching of
Sec. 2.3): a density wave rho = 1 + 0.2 sin(pi (x + y + z - 3 t)) carried by
U = (1, 1, 1) at p = 1, the exact solution of the Euler equations, on
periodic perturbed boxes of tetrahedra, prisms, pyramids and hexahedra.

Initial cell averages and average gradients, and the exact averages at the
final time, come from the analytic wave (by the divergence theorem over the
cells' own faces), not from the method.  With the time step proportional
to the cell size, the L1 error of the density averages falls at third order;
the meshes the oracle finishes in seconds (6 and 12 cells a side) are not
yet fully asymptotic, so the observed order is asserted above 2.5 (measured
2.7 to 2.9).  A scheme that lost an order anywhere (a linear instead of a
quadratic reconstruction, a dropped gradient update, a first-order time
step) would show an order near 2 or below."""
import numpy as np
import pytest

import oracle
import paper_2109_09965_amd.inputs as I
from exact_averages import wave_averages

GAMMA = 1.4


def conserved(rho):
    """Conserved variables of the wave for density values rho: U = (1, 1, 1),
    p = 1, so E = p / (gamma - 1) + 3 rho / 2; rows (rho, rho U, E)."""
    rho = np.asarray(rho)
    return np.stack([rho, rho, rho, rho, 1 / (GAMMA - 1) + 1.5 * rho])


def wave_state(mesh, t):
    """(W [5, n], dW [3, 5, n], cell volumes) of the exact wave at time t:
    the density gradient is the same in each direction."""
    s, c, vol = wave_averages(mesh, np.pi * np.ones(3), 3 * np.pi * t)
    W = conserved(1 + 0.2 * s)
    d = conserved(0.2 * np.pi * c) - conserved(np.zeros_like(c))
    return np.ascontiguousarray(W), np.ascontiguousarray(np.stack([d, d, d])), vol


def wave_error(layer, n, T, scheme, cfl=0.3):
    """L1 error (per unit volume) of the density averages at time T."""
    mesh = I.box3d_mesh((n, n, n), L=(2.0, 2.0, 2.0), layer_types=[layer] * n, periodic=True,
                        perturb=0.15, seed=4)
    W, dW, vol = wave_state(mesh, 0.0)
    om = oracle.Mesh(mesh)
    ce = om.cells()
    assert np.allclose(ce["vol"], vol, rtol=1e-12, atol=0)
    dt0 = cfl * ce["h"].min() / (np.sqrt(3) + np.sqrt(GAMMA / 0.8))
    nst = int(np.ceil(T / dt0))
    s = oracle.Solver(om, oracle.Params(W_inf=conserved(1.0), time_scheme=scheme, explicit_only=1,
                                        dt_fixed=T / nst))
    for _ in range(nst):
        s.cycle(W, dW)
    Wex, _, _ = wave_state(mesh, T)
    return (np.abs(W[0] - Wex[0]) * vol).sum() / vol.sum()


@pytest.mark.parametrize("layer", ["hex", "prism", "pyr", "tet"])
def test_design_order_3d_cells(layer):
    errs = [wave_error(layer, n, 0.1, oracle.S2O4) for n in (6, 12)]
    order = np.log2(errs[0] / errs[1])
    print(f"{layer}: L1 errors {errs}, order {order:.2f}")
    assert order > 2.5, (layer, errs, order)


def test_design_order_3d_s1o2():
    """S1O2 is second order in time; with the time step tied to the cell size
    at this CFL number its time error stays below the third-order spatial
    error, so the observed order matches S2O4's."""
    errs = [wave_error("hex", n, 0.1, oracle.S1O2) for n in (6, 12)]
    order = np.log2(errs[0] / errs[1])
    print(f"S1O2 hex: L1 errors {errs}, order {order:.2f}")
    assert order > 2.5, (errs, order)
