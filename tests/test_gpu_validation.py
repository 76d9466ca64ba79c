"""Converged drag, wake length and separation angle against the values the
paper prints (Sec. 4), through the C ABI, with the no-slip adiabatic wall
of the paper's viscous cases.

These are behavioural checks of the whole method, not parity: the paper's
numbers come from finer meshes than the ones run here, so the tolerance is
the spread of the values printed beside them (the cylinder's experimental
range 1.46-1.56 is about +-3 % around 1.525; the sphere's schemes give
1.002-1.016 and the experiment 1.0).  The cylinder drag of the paper's
conditions must also come out the same on two meshes a factor two apart, to
1 %: a wall treatment that is not consistent shows up as a strong mesh and
Mach dependence of the pressure drag."""
import json
import os

import numpy as np
import pytest

import paper_2109_09965_amd as cg
import paper_2109_09965_amd.inputs as I

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "drag_paper.json")))


def wake_and_separation(m, W, n_theta):
    """Wake length (rear of the cylinder to where the centreline velocity
    turns positive, in diameters) and separation angle (from the rear
    stagnation point, where the first wall layer's tangential velocity
    changes sign), from the converged cell averages of the O-mesh."""
    vol, cen, h = cg.Mesh(m).geometry()
    cen = np.asarray(cen)
    cen = cen if cen.shape[0] == m["n_cell"] else cen.T
    x, y = cen[:, 0], cen[:, 1]
    r, th = np.hypot(x, y), np.arctan2(y, x)
    u, v = W[1] / W[0], W[2] / W[0]
    sel = (np.abs(th) < 2 * np.pi / n_theta) & (x > 0)
    o = np.argsort(r[sel])
    rs, us = r[sel][o], u[sel][o]
    j = np.nonzero((us[:-1] < 0) & (us[1:] >= 0))[0][0]
    wake = rs[j] - us[j] * (rs[j + 1] - rs[j]) / (us[j + 1] - us[j]) - 0.5
    radii = np.unique(np.round(r, 6))
    wall = (r < radii[0] + 0.6 * (radii[2] - radii[0])) & (y > 0)
    tw, uw = th[wall], (-u * np.sin(th) + v * np.cos(th))[wall]
    o = np.argsort(tw)
    tw, uw = tw[o], uw[o]
    j = np.nonzero(np.sign(uw[:-1]) != np.sign(uw[1:]))[0][0]
    sep = np.degrees(tw[j] - uw[j] * (tw[j + 1] - tw[j]) / (uw[j + 1] - uw[j]))
    return wake, sep


def converged_cd(m, Ma, Re, area, max_cycles, state=None):
    w = I.free_stream(m["dim"], Ma)
    b = cg.Batch([cg.Mesh(m)], [cg.Params(W_inf=w, mu=Ma / Re, Pr=0.72, area_ref=area)])
    W, dW = I.uniform_state(m, w)
    b.upload(0, W, dW)
    rep, _ = b.solve(max_cycles=max_cycles, tol=1e-9, check_every=8)
    r = rep[0]
    cd = r["cd"]
    print(f"{m['name'] if 'name' in m else m['dim']}: {r['cycles']} cycles, converged {r['converged']}, "
          f"Cd {cd:.4f}", flush=True)
    assert r["converged"], r
    if state is not None:
        state.append(b.download(0)[0])
    return cd


def test_cylinder_re40_matches_paper():
    g = GOLD["cylinder_re40"]
    cds, states = [], []
    for nt, nr, ratio, h in ((64, 32, 1.1, 0.09695), (128, 64, 1.06, 0.05)):
        m = I.cylinder_mesh(nt, nr, 0.5, ratio=ratio, first_spacing=h, wall=I.BC_NOSLIP_ADIABATIC)
        cds.append(converged_cd(m, g["Ma"], g["Re"], 1.0, 6000, states))
    # the finer mesh (Mesh I's near-wall size): wake length and separation
    # angle within the spread of the values printed beside the paper's
    wake, sep = wake_and_separation(m, states[-1], 128)
    print(f"wake length {wake:.3f} (paper {g['wake_length']}), separation angle {sep:.2f} deg "
          f"(paper {g['separation_angle_deg']})", flush=True)
    assert abs(wake - g["wake_length"]) <= 0.05 * g["wake_length"]
    assert abs(sep - g["separation_angle_deg"]) <= 1.5
    lo, hi = g["Cd_experiment_range"]
    for cd in cds:
        assert lo <= cd <= hi
        assert abs(cd - g["Cd"]) <= 0.03 * g["Cd"]
    assert abs(cds[0] - cds[1]) <= 0.01 * g["Cd"]


def sphere_wake_and_separation(m, W):
    """Closed-wake length along the rear axis (diameters, from the rear of the
    sphere) and separation angle from the front stagnation point, where the
    azimuthal mean of the first wall layer's meridional velocity changes
    sign (2-degree bins)."""
    vol, cen, h = cg.Mesh(m).geometry()
    cen = np.asarray(cen)
    cen = cen if cen.shape[0] == m["n_cell"] else cen.T
    x, rp, r = cen[:, 0], np.hypot(cen[:, 1], cen[:, 2]), np.linalg.norm(cen, axis=1)
    phi = np.arctan2(rp, x)
    u = W[1:4] / W[0]
    sel = (phi < 0.08) & (x > 0.5)
    o = np.argsort(x[sel])
    xs, us = x[sel][o], u[0][sel][o]
    j = np.nonzero((us[:-1] < 0) & (us[1:] >= 0))[0][0]
    wake = xs[j] - us[j] * (xs[j + 1] - xs[j]) / (us[j + 1] - us[j]) - 0.5
    wall = r < r.min() + 0.02
    rq = np.maximum(rp, 1e-30)
    uphi = -np.sin(phi) * u[0] + np.cos(phi) * (u[1] * cen[:, 1] + u[2] * cen[:, 2]) / rq
    bins = np.linspace(0, np.pi, 91)
    idx = np.digitize(phi[wall], bins) - 1
    c, mean = [], []
    for k in range(90):
        if np.any(idx == k):
            c.append(0.5 * (bins[k] + bins[k + 1]))
            mean.append(uphi[wall][idx == k].mean())
    c, mean = np.array(c), np.array(mean)
    j = np.nonzero(np.sign(mean[:-1]) != np.sign(mean[1:]))[0][0]
    sep_rear = c[j] - mean[j] * (c[j + 1] - c[j]) / (mean[j + 1] - mean[j])
    return wake, 180.0 - np.degrees(sep_rear)


def test_sphere_re118_matches_paper():
    g = GOLD["sphere_re118"]
    m = I.sphere_case_mesh()
    states = []
    cd = converged_cd(m, g["Ma"], g["Re"], np.pi * 0.25, 3000, states)
    assert abs(cd - g["Cd"]) <= 0.03 * g["Cd"]
    wake, sep = sphere_wake_and_separation(m, states[0])
    print(f"wake length {wake:.3f} (paper {g['wake_length']}), separation angle {sep:.2f} deg "
          f"(paper {g['separation_angle_deg']})", flush=True)
    assert abs(wake - g["wake_length"]) <= 0.05
    assert abs(sep - g["separation_angle_deg"]) <= 2.5


def test_two_level_cycle_accelerates_steady_convergence():
    """The paper's central observation through the C ABI: on the Re 40
    cylinder the two-level cycle reaches a residual drop of 1e-10, while
    explicit marching at the same CFL, given ten times as many steps, is
    still more than a hundred times short of it."""
    g = GOLD["cylinder_re40"]
    m = I.cylinder_mesh(32, 16, wall=I.BC_NOSLIP_ADIABATIC)
    w = I.free_stream(2, g["Ma"])
    lm = cg.Mesh(m)
    drops = {}
    for expl in (0, 1):
        b = cg.Batch([lm], [cg.Params(W_inf=w, mu=g["Ma"] / g["Re"], Pr=0.72, explicit_only=expl)])
        W, dW = I.uniform_state(m, w)
        b.upload(0, W, dW)
        cycles = 4000 if not expl else 10 * drops[0][0]
        rep, h = b.solve(max_cycles=cycles, tol=1e-10 if not expl else 0.0, check_every=8, history=True)
        r = rep[0]
        hh = h[0][:r["cycles"]]
        drops[expl] = (r["cycles"], hh[-1] / hh[0])
        print(f"explicit_only={expl}: {r['cycles']} cycles, residual drop {hh[-1] / hh[0]:.2e}", flush=True)
    assert drops[0][1] <= 1e-10
    assert drops[1][1] > 1e-8, drops


@pytest.mark.parametrize("scheme", [cg.S1O2, cg.S2O4])
def test_low_level_flux_choice(scheme):
    """Sec. 4 (cylinder): KFVS and Lax-Friedrichs on the low level converge
    alike.  Under S1O2 the transferred residual R1 is exactly the explicit
    step's increment over dt, so the cycle can only stand still where R1 = 0:
    the converged state is the same for both low-level fluxes (to the residual
    level reached).  Under S2O4 the step's increment and R1 vanish at states
    that differ at O(dt^2); the cycle stands still where the correction
    cancels the increment, which depends slightly on the low-level operator."""
    g = GOLD["cylinder_re40"]
    m = I.cylinder_mesh(64, 32, 0.5, ratio=1.1, first_spacing=0.09695, wall=I.BC_NOSLIP_ADIABATIC)
    w = I.free_stream(2, g["Ma"])
    lm = cg.Mesh(m)
    out = {}
    for lf in (cg.LOW_KFVS, cg.LOW_LF):
        b = cg.Batch([lm], [cg.Params(W_inf=w, mu=g["Ma"] / g["Re"], Pr=0.72, low_flux=lf, time_scheme=scheme,
                                      area_ref=1.0)])
        W, dW = I.uniform_state(m, w)
        b.upload(0, W, dW)
        rep, _ = b.solve(max_cycles=6000, tol=1e-12, check_every=8)
        r = rep[0]
        out[lf] = (r["cycles"], b.download(0)[0], r["cd"])
        print(f"scheme {scheme} low flux {lf}: {r['cycles']} cycles, converged {r['converged']}, "
              f"Cd {out[lf][2]:.8f}", flush=True)
        assert r["converged"], r
    (ck, Wk, cdk), (cl, Wl, cdl) = out[cg.LOW_KFVS], out[cg.LOW_LF]
    dw = np.abs(Wk - Wl).max() / np.abs(Wk).max()
    print(f"state difference {dw:.2e}, Cd difference {abs(cdk - cdl):.2e}", flush=True)
    if scheme == cg.S1O2:
        assert dw <= 1e-9 and abs(cdk - cdl) <= 1e-8
    else:
        assert dw <= 1e-4 and abs(cdk - cdl) <= 1e-4 * cdk
    assert 0.5 <= cl / ck <= 2.0
