"""Captured cycles (HIP graphs) and batches of cases (GPU).

A graph replay must reproduce the eager cycles bit for bit, replay after
replay, with unrelated eager device work and synchronisations in between.
A case stepped inside a batch of uneven cases must give bitwise the same
state as the same case stepped alone (per-case reductions have a fixed
shape and never mix cases)."""
import numpy as np
import pytest

import oracle
import paper_2109_09965_amd as cg
import paper_2109_09965_amd.inputs as I

pytestmark = pytest.mark.gpu


def case(kind, seed):
    if kind == "cyl":
        m = I.cylinder_mesh(32, 16, wall=I.BC_NOSLIP_ISOTHERMAL)
        Winf = I.free_stream(2, 0.15 + 0.05 * seed, 2.0 * seed)
        kw = dict(W_inf=Winf, mu=0.15 / 40, Pr=0.72)
    elif kind == "cyl_small":
        m = I.cylinder_mesh(24, 12)
        Winf = I.free_stream(2, 0.3, -3.0)
        kw = dict(W_inf=Winf)
    elif kind == "sphere":
        m = I.sphere_mesh(8, 16, 8, 3, 2)
        Winf = I.free_stream(3, 0.25)
        kw = dict(W_inf=Winf, mu=0.0025, Pr=0.72)
    elif kind == "sphere_b":
        m = I.sphere_mesh(6, 12, 7, 2, 3)
        Winf = I.free_stream(3, 0.35, 5.0)
        kw = dict(W_inf=Winf, mu=0.004, Pr=0.72)
    W, dW = I.smooth_state(m, Winf, seed=seed, amp=0.03)
    return m, kw, W, dW


@pytest.mark.parametrize("kind", ["cyl", "sphere"])
def test_graph_replays_match_eager(kind):
    import torch
    m, kw, W, dW = case(kind, 1)
    eager = cg.Batch([cg.Mesh(m)], [cg.Params(**kw)])
    graph = cg.Batch([cg.Mesh(m)], [cg.Params(**kw)])
    eager.upload(0, W, dW)
    graph.upload(0, W, dW)
    n = 3
    graph.graph_create(n)
    hist = torch.zeros(n, dtype=torch.float64, device="cuda")
    res = torch.zeros(1, dtype=torch.float64, device="cuda")
    for rep in range(3):
        graph.graph_launch(hist)
        ref = []
        for _ in range(n):
            eager.cycle(res)
            ref.append(float(res.cpu()[0]))
        # unrelated eager work and a synchronisation between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        torch.cuda.synchronize()
        Wg, dWg = graph.download(0)
        We, dWe = eager.download(0)
        assert np.array_equal(Wg, We) and np.array_equal(dWg, dWe), rep
        assert np.array_equal(hist.cpu().numpy(), np.array(ref)), rep


def test_graph_matches_oracle():
    import torch
    m, kw, W, dW = case("cyl", 2)
    b = cg.Batch([cg.Mesh(m)], [cg.Params(**kw)])
    b.upload(0, W, dW)
    s = oracle.Solver(oracle.Mesh(m), oracle.Params(**kw))
    b.graph_create(4)
    b.graph_launch()
    for _ in range(4):
        s.cycle(W, dW)
    Wg, _ = b.download(0)
    assert np.abs(Wg - W).max() <= 1e-11 * np.abs(W).max()


@pytest.mark.parametrize("kinds", [["cyl", "cyl_small", "cyl"], ["sphere", "sphere_b"]])
def test_batch_equals_alone(kinds):
    import torch
    cases = [case(k, i) for i, k in enumerate(kinds)]
    meshes = [cg.Mesh(c[0]) for c in cases]
    batch = cg.Batch(meshes, [cg.Params(**c[1]) for c in cases])
    alone = [cg.Batch([cg.Mesh(c[0])], [cg.Params(**c[1])]) for c in cases]
    for i, c in enumerate(cases):
        batch.upload(i, c[2], c[3])
        alone[i].upload(0, c[2], c[3])
    rb = torch.zeros(len(cases), dtype=torch.float64, device="cuda")
    ra = torch.zeros(1, dtype=torch.float64, device="cuda")
    for k in range(3):
        batch.cycle(rb)
        for i in range(len(cases)):
            alone[i].cycle(ra)
            assert float(rb.cpu()[i]) == float(ra.cpu()[0]), (k, i)
    for i in range(len(cases)):
        Wb, dWb = batch.download(i)
        Wa, dWa = alone[i].download(0)
        assert np.array_equal(Wb, Wa) and np.array_equal(dWb, dWa), i


def test_batch_against_oracle():
    kinds = ["cyl", "cyl_small"]
    cases = [case(k, i) for i, k in enumerate(kinds)]
    batch = cg.Batch([cg.Mesh(c[0]) for c in cases], [cg.Params(**c[1]) for c in cases])
    for i, c in enumerate(cases):
        batch.upload(i, c[2], c[3])
    for _ in range(2):
        batch.cycle()
    for i, (m, kw, W, dW) in enumerate(cases):
        s = oracle.Solver(oracle.Mesh(m), oracle.Params(**kw))
        W, dW = W.copy(), dW.copy()
        for _ in range(2):
            s.cycle(W, dW)
        Wb, _ = batch.download(i)
        assert np.abs(Wb - W).max() <= 1e-11 * np.abs(W).max(), i


def test_solve_freezes_converged_cases():
    """cgks_solve stops updating a case once it meets its tolerance while the
    others keep cycling."""
    kinds = ["cyl", "cyl_small"]
    cases = [case(k, i) for i, k in enumerate(kinds)]
    batch = cg.Batch([cg.Mesh(c[0]) for c in cases], [cg.Params(**c[1]) for c in cases])
    for i, c in enumerate(cases):
        batch.upload(i, c[2], c[3])
    rep, hist = batch.solve(max_cycles=40, tol=0.5, check_every=1, history=True)
    assert all(r["cycles"] >= 1 for r in rep)
    first_done = min(range(2), key=lambda i: rep[i]["cycles"])
    if rep[first_done]["converged"]:
        n = rep[first_done]["cycles"]
        W1, _ = batch.download(first_done)
        batch.solve(max_cycles=1, tol=0.0, check_every=1)   # every case active again
        W2, _ = batch.download(first_done)
        assert not np.array_equal(W1, W2)


def test_solve_reports_the_cycles_the_state_ran():
    """With checks every 8 cycles (run as captured graphs) a case that meets
    its tolerance inside a block stops at the check that ends the block: the
    report counts those cycles, the history holds each of them, and the state
    equals the case stepped eagerly for that many cycles, bitwise."""
    m, kw, W, dW = case("cyl", 0)
    lm = cg.Mesh(m)
    b = cg.Batch([lm], [cg.Params(**kw)])
    b.upload(0, W, dW)
    _, href = b.solve(max_cycles=64, tol=0.0, check_every=1, history=True)
    ratio = href[0] / href[0][0]
    # a new running minimum of Res reached strictly inside a block of 8
    met = next(c for c in range(9, 60) if c % 8 and ratio[c - 1] < ratio[:c - 1].min())
    tol = ratio[met - 1]
    b.upload(0, W, dW)
    rep, hist = b.solve(max_cycles=64, tol=tol, check_every=8, history=True)
    r = rep[0]
    assert r["converged"] and r["cycles"] == 8 * (met // 8 + 1), (met, r)
    np.testing.assert_array_equal(hist[0][:r["cycles"]], href[0][:r["cycles"]])
    assert r["res_last"] == href[0][r["cycles"] - 1]
    Ws, dWs = b.download(0)
    e = cg.Batch([lm], [cg.Params(**kw)])
    e.upload(0, W, dW)
    for _ in range(r["cycles"]):
        e.cycle()
    We, dWe = e.download(0)
    assert np.array_equal(Ws, We) and np.array_equal(dWs, dWe)


@pytest.mark.parametrize("kinds,precision", [(["cyl", "cyl_small", "cyl"], cg.FP64), (["sphere", "sphere_b"], cg.FP64),
                                             (["sphere", "sphere_b"], cg.MIXED32)])
def test_autotuned_batch_steps_bitwise_like_untuned(kinds, precision):
    """Tuning picks launch shapes only: the tuned batch's states equal the
    untuned batch's bitwise, and the picks are among the candidates."""
    cases = [case(k, i) for i, k in enumerate(kinds)]
    tuned = cg.Batch([cg.Mesh(c[0]) for c in cases], [cg.Params(**c[1]) for c in cases], precision=precision)
    plain = cg.Batch([cg.Mesh(c[0]) for c in cases], [cg.Params(**c[1]) for c in cases], precision=precision)
    for i, c in enumerate(cases):
        tuned.upload(i, c[2], c[3])
        plain.upload(i, c[2], c[3])
    picks = tuned.autotune()
    print(picks, flush=True)
    assert picks["sweep_chunk"] in (16, 32, 64)
    assert all(picks[k] in (64, 128, 256) for k in ("flux_block", "cell_block", "low_face_block", "low_cell_block"))
    for _ in range(3):
        tuned.cycle()
        plain.cycle()
    for i in range(len(cases)):
        Wt, dWt = tuned.download(i)
        Wp, dWp = plain.download(i)
        assert np.array_equal(Wt, Wp) and np.array_equal(dWt, dWp), i


def test_nonphysical_case_is_flagged_and_leaves_the_batch_alone():
    """A case whose state has a cell of negative pressure is reported
    non-physical after its first cycle and frozen, while the other case of
    the batch runs on and ends bitwise equal to the same case run alone: a
    bad case never fails a batch (per-case flags, time steps and norms)."""
    good, bad = case("cyl", 0), case("cyl_small", 1)
    Wb = bad[2].copy()
    rho, mom = Wb[0, 7], Wb[1:3, 7]
    Wb[-1, 7] = 0.25 * 0.5 * float(mom @ mom) / rho      # E below the kinetic energy: p < 0
    assert 0.4 * (Wb[-1, 7] - 0.5 * float(mom @ mom) / rho) < 0
    b = cg.Batch([cg.Mesh(good[0]), cg.Mesh(bad[0])], [cg.Params(**good[1]), cg.Params(**bad[1])])
    b.upload(0, good[2], good[3])
    b.upload(1, Wb, bad[3])
    rep, _ = b.solve(max_cycles=6, tol=0.0, check_every=1)
    print(rep, flush=True)
    assert rep[1]["status"] == cg.ENONPHYS and rep[1]["cycles"] == 1 and not rep[1]["converged"]
    assert rep[0]["status"] == cg.ENOTCONV and rep[0]["cycles"] == 6
    Wg, dWg = b.download(0)
    a = cg.Batch([cg.Mesh(good[0])], [cg.Params(**good[1])])
    a.upload(0, good[2], good[3])
    for _ in range(6):
        a.cycle()
    Wa, dWa = a.download(0)
    assert np.array_equal(Wg, Wa) and np.array_equal(dWg, dWa)
