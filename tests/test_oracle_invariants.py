"""Method-level pins of the oracle (CPU only): free-stream preservation,
discrete conservation, the closed forms of the time marching, the S1O2
residual identity behind the multigrid fixed point, and the design order
of accuracy on a smooth solution."""
import numpy as np
import pytest

import oracle
import paper_2109_09965_amd.inputs as I


def run_cycles(mesh, params, W, dW, n):
    s = oracle.Solver(oracle.Mesh(mesh), params)
    res = [s.cycle(W, dW) for _ in range(n)]
    return s, res


@pytest.mark.parametrize("mk,mach,aoa,mu,Pr", [
    (lambda: I.cylinder_mesh(32, 16, wall=I.BC_FARFIELD), 0.2, 3.0, 0.0, 1.0),
    (lambda: I.sphere_mesh(8, 16, 8, 3, 2, wall=I.BC_FARFIELD), 0.25, 10.0, 0.01, 0.72),
    (lambda: I.box2d_mesh(8, perturb=0.3, seed=2), 0.5, 30.0, 0.02, 0.72),
    (lambda: I.box3d_mesh((3, 3, 5), periodic=True, perturb=0.2, seed=4), 0.4, 20.0, 0.01, 0.72),
])
@pytest.mark.parametrize("low_flux", [oracle.LOW_KFVS, oracle.LOW_LF])
def test_free_stream_is_preserved(mk, mach, aoa, mu, Pr, low_flux):
    mesh = mk()
    d = mesh["dim"]
    Winf = I.free_stream(d, mach, aoa)
    W, dW = I.uniform_state(mesh, Winf)
    _, res = run_cycles(mesh, oracle.Params(W_inf=Winf, mu=mu, Pr=Pr, low_flux=low_flux), W, dW, 20)
    assert np.abs(W - Winf[:, None]).max() <= 1e-13
    assert np.abs(dW).max() <= 1e-12
    assert max(res) <= 1e-14


@pytest.mark.parametrize("mk", [lambda: I.box2d_mesh(8, perturb=0.3, seed=2),
                                lambda: I.box3d_mesh((3, 3, 5), periodic=True, perturb=0.2, seed=4)])
@pytest.mark.parametrize("scheme,low_flux", [(oracle.S2O4, oracle.LOW_KFVS), (oracle.S1O2, oracle.LOW_KFVS),
                                             (oracle.S2O4, oracle.LOW_LF)])
def test_periodic_conservation(mk, scheme, low_flux):
    """Each face flux enters its two cells with opposite signs: the high-order
    stages conserve sum |V| W and the residuals of both levels (KFVS or
    Lax-Friedrichs on the low one) sum to zero."""
    mesh = mk()
    d = mesh["dim"]
    Winf = I.free_stream(d, 0.3, 15.0)
    W, dW = I.smooth_state(mesh, Winf, seed=3, amp=0.05)
    om = oracle.Mesh(mesh)
    vol = om.cells()["vol"]
    s = oracle.Solver(om, oracle.Params(W_inf=Winf, mu=0.01, Pr=0.72, time_scheme=scheme, low_flux=low_flux))
    tot0 = W @ vol
    s.stage(0, W, dW)
    np.testing.assert_allclose(W @ vol, tot0, rtol=1e-14, atol=1e-14)
    if scheme == oracle.S2O4:
        s.stage(1, W, dW)
        np.testing.assert_allclose(W @ vol, tot0, rtol=1e-14, atol=1e-14)
    R1 = s.residual_high(W, dW)
    R0 = s.residual_low(W)
    assert np.abs(R1.sum(1)).max() <= 1e-13 * np.abs(R1).sum()
    assert np.abs(R0.sum(1)).max() <= 1e-13 * np.abs(R0).sum()


@pytest.mark.parametrize("mk,bc", [
    (lambda bc: I.box2d_mesh(8, periodic=False, perturb=0.3, seed=2, bc=bc), I.BC_SLIP_WALL),
    (lambda bc: I.box3d_mesh((3, 3, 5), perturb=0.2, seed=4, bc=bc), I.BC_SLIP_WALL),
    (lambda bc: I.box3d_mesh((3, 3, 5), perturb=0.2, seed=4, bc=bc), I.BC_NOSLIP_ISOTHERMAL),
    (lambda bc: I.box2d_mesh(8, periodic=False, perturb=0.3, seed=2, bc=bc), I.BC_NOSLIP_ADIABATIC),
    (lambda bc: I.box3d_mesh((3, 3, 5), perturb=0.2, seed=4, bc=bc), I.BC_NOSLIP_ADIABATIC),
])
def test_walls_carry_no_mass(mk, bc):
    """A closed box with slip walls conserves mass and energy in the
    high-order stages (the mirrored interface state has no normal mass or
    energy flux); with no-slip isothermal walls mass is conserved.  With
    no-slip adiabatic walls mass and energy are conserved: the wall state
    has zero velocity, so the viscous stress does no work, and the mirrored
    gradients give zero normal temperature derivative, so no heat crosses;
    a wrong sign in the mirrored gradients leaves a heat flux and fails
    this."""
    mesh = mk(bc)
    d = mesh["dim"]
    Winf = I.free_stream(d, 0.3, 15.0)
    W, dW = I.smooth_state(mesh, Winf, seed=5, amp=0.05)
    om = oracle.Mesh(mesh)
    vol = om.cells()["vol"]
    s = oracle.Solver(om, oracle.Params(W_inf=Winf, mu=0.01, Pr=0.72))
    tot0 = W @ vol
    s.stage(0, W, dW)
    s.stage(1, W, dW)
    tot = W @ vol
    assert tot[0] == pytest.approx(tot0[0], rel=1e-14)
    if bc in (I.BC_SLIP_WALL, I.BC_NOSLIP_ADIABATIC):
        assert tot[-1] == pytest.approx(tot0[-1], rel=1e-14)
    R1 = s.residual_high(W, dW)
    assert abs(R1[0].sum()) <= 1e-13 * np.abs(R1[0]).sum()


def open_top_box(mesh, top):
    """The box's boundary faces on the plane x[d-1] = top become far field."""
    d = mesh["dim"]
    ptr, fv, xyz = mesh["face_vert_ptr"], mesh["face_vert"], mesh["xyz"]
    bc = mesh["face_bc"].copy()
    for f in np.nonzero(mesh["face_neigh"] < 0)[0]:
        if np.allclose(xyz[fv[ptr[f]:ptr[f + 1]], d - 1], top):
            bc[f] = I.BC_FARFIELD
    out = dict(mesh)
    out["face_bc"] = bc
    return out


@pytest.mark.parametrize("mk,top,area", [
    (lambda bc: I.box2d_mesh(6, periodic=False, perturb=0.3, seed=3, bc=bc), 2.0, 2.0),
    (lambda bc: I.box3d_mesh((3, 3, 5), perturb=0.2, seed=6, bc=bc), 1.0, 1.0),
])
@pytest.mark.parametrize("bc", [I.BC_SLIP_WALL, I.BC_NOSLIP_ISOTHERMAL, I.BC_NOSLIP_ADIABATIC])
def test_wall_force_of_gas_at_rest_in_an_open_box(mk, top, area, bc):
    """Gas at rest at the free-stream pressure in a box whose top side is
    far field and whose other sides are walls: the wall momentum flux is
    the pressure alone and the walls form a closed surface less the top,
    so the force on them is -p0 * (top area) * e_top, to round-off.  Also
    pins the sign (force of the gas on the walls) and that far-field faces
    do not count."""
    mesh = open_top_box(mk(bc), top)
    d = mesh["dim"]
    Winf = I.free_stream(d, 0.0)
    W, dW = I.uniform_state(mesh, Winf)
    s = oracle.Solver(oracle.Mesh(mesh), oracle.Params(W_inf=Winf, mu=0.01, Pr=0.72))
    s.stage(0, W, dW)
    p0 = 1.0 / 1.4
    expect = np.zeros(d)
    expect[-1] = -p0 * area
    np.testing.assert_allclose(s.force()[:d], expect, rtol=0, atol=1e-13)


@pytest.mark.parametrize("z", [-0.9, -0.3, 0.05, 0.5, 1.2])
def test_time_marching_closed_forms(z):
    """y' = lam y with L = lam y and L_t = lam^2 y: S2O4 reproduces the
    fourth-order Taylor polynomial, S1O2 the second-order one."""
    lam, y, dt = 1.7, 1.3, z / 1.7
    ys = oracle.stage_combine(oracle.S2O4, 0, dt, y, lam * y, lam * lam * y)
    y1 = oracle.stage_combine(oracle.S2O4, 1, dt, y, lam * y, lam * lam * y, lam * lam * ys)
    assert y1 == pytest.approx(y * (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24), rel=1e-14)
    y2 = oracle.stage_combine(oracle.S1O2, 0, dt, y, lam * y, lam * lam * y)
    assert y2 == pytest.approx(y * (1 + z + z * z / 2), rel=1e-14)


@pytest.mark.parametrize("z", [-0.9, -0.3, 0.05, 0.5, 1.2])
def test_gradient_time_update_closed_forms(z):
    """Gradients advance with the interface values they are summed from: for
    an interface value y' = lam y (G = y, Gt = lam y at the start, Gt* = lam
    times the mid-stage value), S2O4's midpoint rule gives the second-order
    Taylor polynomial and S1O2's step the first-order one."""
    lam, y, dt = 1.7, 1.3, z / 1.7
    ys = oracle.grad_combine(oracle.S2O4, 0, dt, 0.0, y, lam * y)
    assert ys == pytest.approx(y * (1 + z / 2), rel=1e-14)
    y1 = oracle.grad_combine(oracle.S2O4, 1, dt, y, ys, lam * ys)
    assert y1 == pytest.approx(y * (1 + z + z * z / 2), rel=1e-14)
    y2 = oracle.grad_combine(oracle.S1O2, 0, dt, 0.0, y, lam * y)
    assert y2 == pytest.approx(y * (1 + z), rel=1e-14)


@pytest.mark.parametrize("mk", [lambda: I.cylinder_mesh(32, 16), lambda: I.sphere_mesh(6, 12, 6, 2, 2)])
@pytest.mark.parametrize("low_flux", [oracle.LOW_KFVS, oracle.LOW_LF])
def test_s1o2_residual_is_the_step_increment(mk, low_flux):
    """R1 is the time-averaged net flux over one step, so with one time step
    |V|^-1 dt R1 is exactly the S1O2 increment from the same state.  Hence a
    state the explicit S1O2 scheme leaves unchanged has R1 = 0, the forcing
    makes the low level start at its own steady state and the correction
    vanishes: the multigrid fixed point is the explicit one."""
    mesh = mk()
    d = mesh["dim"]
    Winf = I.free_stream(d, 0.2, 5.0)
    W, dW = I.smooth_state(mesh, Winf, seed=7, amp=0.03)
    om = oracle.Mesh(mesh)
    vol = om.cells()["vol"]
    P = oracle.Params(W_inf=Winf, mu=0.01 if d == 3 else 0.0, Pr=0.72, time_scheme=oracle.S1O2, dt_fixed=2e-3,
                      low_flux=low_flux)
    s = oracle.Solver(om, P)
    W1, dW1 = W.copy(), dW.copy()
    s.stage(0, W1, dW1)
    R1 = s.residual_high(W, dW)
    np.testing.assert_allclose(W1 - W, P.dt_fixed * R1 / vol, rtol=0, atol=1e-15 * np.abs(W).max())
    # with R1 = 0 the forcing is S = -R0(W): the first implicit step has a
    # zero right-hand side and the correction vanishes
    Wl = W.copy()
    s.lowlevel(Wl, np.zeros_like(W))
    np.testing.assert_allclose(Wl, W, rtol=0, atol=1e-14)


@pytest.mark.parametrize("low_flux", [oracle.LOW_KFVS, oracle.LOW_LF])
def test_low_level_residual_diffuses_a_density_bump_at_rest(low_flux):
    """Gas at rest at uniform pressure with a density bump: the Euler flux
    carries no mass, so the first-order mass residual is the flux's
    numerical dissipation alone.  Both low-level fluxes must move mass from
    the densest cell to its neighbours and into the least dense cell (a wrong
    sign of the dissipation term turns this around), and Lax-Friedrichs
    (dissipation lam_f >= c, the sound speed) more strongly than KFVS
    (whose mass dissipation at rest is sqrt(theta / 2 pi) < c per side)."""
    mesh = I.box2d_mesh(10, perturb=0.2, seed=5)
    om = oracle.Mesh(mesh)
    x = om.cells()["ctr"]
    n = mesh["n_cell"]
    rho = 1.0 + 0.2 * np.exp(-((x[:, 0] - 1.0) ** 2 + (x[:, 1] - 1.0) ** 2) / 0.1)
    W = np.zeros((4, n))
    W[0] = rho
    W[3] = (1.0 / 1.4) / 0.4
    out = {}
    for lf in (oracle.LOW_KFVS, oracle.LOW_LF):
        s = oracle.Solver(om, oracle.Params(W_inf=I.free_stream(2, 0.0), low_flux=lf))
        out[lf] = s.residual_low(W)
    R = out[low_flux]
    imax, imin = int(np.argmax(rho)), int(np.argmin(rho))
    assert R[0, imax] < 0 < R[0, imin]
    assert abs(R[0].sum()) <= 1e-14 * np.abs(R[0]).sum()
    assert np.abs(out[oracle.LOW_LF][0, imax]) > np.abs(out[oracle.LOW_KFVS][0, imax])


def tri_cell_vertices(mesh):
    """Vertex coordinates of each triangle (2-D), neighbour copies shifted."""
    n = mesh["n_cell"]
    pts = [[] for _ in range(n)]
    ptr, fv = mesh["face_vert_ptr"], mesh["face_vert"]
    for f in range(len(mesh["face_owner"])):
        X = mesh["xyz"][fv[ptr[f]:ptr[f + 1]]]
        pts[mesh["face_owner"][f]].extend(list(X))
        nb = mesh["face_neigh"][f]
        if nb >= 0:
            pts[nb].extend(list(X - mesh["face_shift"][f]))
    out = np.zeros((n, 3, 2))
    for i in range(n):
        P = np.unique(np.round(np.array(pts[i]), 12), axis=0)
        assert len(P) == 3
        out[i] = P
    return out


def tri_average(P, fn, nq=8):
    """Exact-to-high-degree cell averages over triangles (collapsed Gauss)."""
    x, w = np.polynomial.legendre.leggauss(nq)
    x, w = 0.5 * (x + 1), 0.5 * w
    s, t = np.meshgrid(x, x, indexing="ij")
    ws = np.outer(w, w) * (1 - s)
    a, b = s, t * (1 - s)
    X = (P[:, 0, None, None, :] * (1 - a - b)[None, :, :, None] + P[:, 1, None, None, :] * a[None, :, :, None]
         + P[:, 2, None, None, :] * b[None, :, :, None])
    v = fn(X)
    return (v * ws[None, ..., None]).sum((1, 2)) / ws.sum() if v.ndim == 4 else (v * ws[None]).sum((1, 2)) / ws.sum()


def wave_fields(X, t=0.0):
    """rho = 1 + 0.2 sin(pi (x + y - 2t)), U = (1, 1), p = 1 as (W, dW)."""
    ph = np.pi * (X[..., 0] + X[..., 1] - 2 * t)
    rho = 1 + 0.2 * np.sin(ph)
    dr = 0.2 * np.pi * np.cos(ph)
    W = np.stack([rho, rho, rho, 1 / 0.4 + rho], -1)
    dWx = np.stack([dr, dr, dr, dr], -1)
    return W, dWx


@pytest.mark.parametrize("scheme", [oracle.S2O4])
def test_design_order_density_wave(scheme):
    """One period of a density wave on perturbed periodic triangle meshes:
    the L1 error of the cell averages falls at third order."""
    errs = []
    for n in (8, 16, 32):
        mesh = I.box2d_mesh(n, L=2.0, periodic=True, perturb=0.2, seed=3)
        P = tri_cell_vertices(mesh)
        Wav = tri_average(P, lambda X: wave_fields(X)[0])
        dav = tri_average(P, lambda X: wave_fields(X)[1])
        W = np.ascontiguousarray(Wav.T)
        dW = np.ascontiguousarray(np.stack([dav.T, dav.T]))
        om = oracle.Mesh(mesh)
        ce = om.cells()
        dt0 = 0.3 * ce["h"].min() / (np.sqrt(2) + np.sqrt(1.4 / 0.8))
        nst = int(np.ceil(1.0 / dt0))
        s = oracle.Solver(om, oracle.Params(W_inf=np.array([1, 1, 1, 3.5]), time_scheme=scheme, explicit_only=1,
                                            dt_fixed=1.0 / nst))
        for _ in range(nst):
            s.cycle(W, dW)
        err = (np.abs(W[0] - Wav[:, 0]) * ce["vol"]).sum() / 4.0
        errs.append(err)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > 2.6, (errs, orders)


def test_multigrid_accelerates_viscous_cylinder():
    """Steady viscous cylinder (Re 40, Ma 0.15, no-slip isothermal wall):
    the two-level cycle drives the density residual down far faster per
    cycle than explicit marching alone, the paper's central observation."""
    mesh = I.cylinder_mesh(32, 16, wall=I.BC_NOSLIP_ISOTHERMAL)
    Ma, Re = 0.15, 40.0
    Winf = I.free_stream(2, Ma)
    drops = {}
    for expl in (0, 1):
        W, dW = I.uniform_state(mesh, Winf)
        s = oracle.Solver(oracle.Mesh(mesh), oracle.Params(W_inf=Winf, mu=Ma / Re, Pr=0.72,
                                                           time_scheme=oracle.S1O2, explicit_only=expl))
        res = [s.cycle(W, dW) for _ in range(150)]
        drops[expl] = res[-1] / res[0]
    assert drops[0] < 1e-4
    assert drops[0] < 1e-2 * drops[1], drops


@pytest.mark.parametrize("dim", [2, 3])
def test_low_level_mass_fluxes_at_rest_match_closed_forms(dim):
    """Gas at rest at uniform pressure p, inviscid, with the density of one
    cell i raised: across a face of i only the numerical dissipation moves
    mass, so each neighbour j's first-order mass residual (the face sum, not
    divided by the volume) is S_f times the mass flux from i to j, and i's is
    minus the sum over its faces.
    Closed forms, independent of the oracle's code:
      KFVS: the one-sided mass flux of a Maxwellian at rest is
            rho sqrt(theta / 2 pi) = sqrt(rho p / 2 pi) (kinetic theory), so
            the flux is sqrt(p / 2 pi) (sqrt(rho_i) - sqrt(rho_j));
      Lax-Friedrichs: 1/2 lam_f (rho_i - rho_j) with lam_f the larger of the
            two sides' spectral radii of the Euler flux Jacobian, |U.n| + c
            = c = sqrt(gamma p / rho) at rest (the lighter side here).
    This pins the inviscid part of the implicit operator's spectral radius
    and the max-of-sides rule."""
    if dim == 2:
        mesh = I.box2d_mesh(6, perturb=0.0, seed=1)
    else:
        mesh = I.box3d_mesh((4, 4, 4), periodic=True)
    om = oracle.Mesh(mesh)
    S = om.faces()["S"]
    own, nb = np.asarray(mesh["face_owner"]), np.asarray(mesh["face_neigh"])
    n, g, p = mesh["n_cell"], 1.4, 0.7
    i = n // 2
    fi = np.flatnonzero((own == i) | (nb == i))
    assert len(fi) >= dim + 1 and (nb[fi] >= 0).all()
    rho_i, rho_0 = 1.3, 1.0
    W = np.zeros((dim + 2, n))
    W[0] = rho_0
    W[0, i] = rho_i
    W[dim + 1] = p / (g - 1.0)
    flux = {oracle.LOW_KFVS: np.sqrt(p / (2 * np.pi)) * (np.sqrt(rho_i) - np.sqrt(rho_0)),
            oracle.LOW_LF: 0.5 * np.sqrt(g * p / rho_0) * (rho_i - rho_0)}
    for lf, F in flux.items():
        s = oracle.Solver(om, oracle.Params(W_inf=I.free_stream(dim, 0.0), mu=0.0, gamma=g, low_flux=lf))
        R = s.residual_low(W)
        for f in fi:
            j = nb[f] if own[f] == i else own[f]
            assert R[0, j] == pytest.approx(S[f] * F, rel=1e-12), (lf, f)
        assert R[0, i] == pytest.approx(-S[fi].sum() * F, rel=1e-12), lf
