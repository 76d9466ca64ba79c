"""Pools: batches with fixed capacity that admit and release cases while
others keep running (continuous batching).

A case must give bitwise the same state in a pool, with other cases
admitted and released around it, as alone in its own batch: reductions and
sweep blocks never span two cases and their shapes depend only on the case.
Admission is bounded by the pool's capacity (its HBM footprint) and freed
ranges are reused."""
import numpy as np
import pytest

import oracle
import paper_2109_09965_amd as cg
import paper_2109_09965_amd.inputs as I

pytestmark = pytest.mark.gpu


def cyl(n_theta, mach, aoa, seed):
    m = I.cylinder_mesh(n_theta, n_theta // 2)
    w = I.free_stream(2, mach, aoa)
    W, dW = I.smooth_state(m, w, seed=seed, amp=0.02)
    return m, cg.Params(W_inf=w), W, dW


def counts(lm):
    return lm.n_cell, lm.n_face, lm.n_gp, lm.info.n_boundary_face


def alone(m, p, W, dW, n, precision=cg.FP64):
    b = cg.Batch([cg.Mesh(m)], [p], precision=precision)
    b.upload(0, W, dW)
    for _ in range(n):
        b.cycle()
    return b.download(0)


@pytest.mark.parametrize("precision", [cg.FP64, cg.MIXED32])
def test_case_in_a_changing_pool_equals_alone(precision):
    A = cyl(32, 0.2, 2.0, 1)
    B = cyl(48, 0.3, -1.0, 2)
    C = cyl(16, 0.25, 0.5, 3)
    D = cyl(24, 0.15, 4.0, 4)
    lms = {k: cg.Mesh(v[0]) for k, v in dict(A=A, B=B, C=C, D=D).items()}
    tot = np.sum([counts(lm) for lm in lms.values()], axis=0)
    pool = cg.Batch.pool(2, 3, *[int(x) for x in tot], precision=precision)
    sa = pool.admit(lms["A"], A[1])
    pool.upload(sa, A[2], A[3])
    sb = pool.admit(lms["B"], B[1])
    pool.upload(sb, B[2], B[3])
    pool.cycle()                      # A: 1
    sc = pool.admit(lms["C"], C[1])
    pool.upload(sc, C[2], C[3])
    pool.cycle()                      # A: 2, C: 1
    pool.release(sb)                  # B leaves; D takes (part of) its ranges
    sd = pool.admit(lms["D"], D[1])
    pool.upload(sd, D[2], D[3])
    assert pool.cell_off[sd] >= 0
    pool.cycle()                      # A: 3, C: 2, D: 1
    pool.cycle()                      # A: 4, C: 3, D: 2
    for name, case, slot, n in (("A", A, sa, 4), ("C", C, sc, 3), ("D", D, sd, 2)):
        Wp, dWp = pool.download(slot)
        Wa, dWa = alone(case[0], case[1], case[2], case[3], n, precision)
        print(f"{name}: max |pool - alone| W {np.abs(Wp - Wa).max():.1e}", flush=True)
        assert np.array_equal(Wp, Wa) and np.array_equal(dWp, dWa), name


@pytest.mark.parametrize("precision", [cg.FP64, cg.MIXED32])
def test_tiled_cases_in_a_changing_pool_equal_alone(precision):
    """Meshes cut into many ragged tiles (sweep runs per tile and colour,
    faces in their cells' order) admitted and released around each other:
    each case still equals itself alone in one whole-mesh tile, bitwise."""
    A = cyl(32, 0.2, 2.0, 7)
    m3 = I.cubed_sphere_mesh(4, 8, 3, 2)
    w3 = I.free_stream(3, 0.3, 3.0)
    W3, dW3 = I.smooth_state(m3, w3, seed=8, amp=0.02)
    S3 = (m3, cg.Params(W_inf=w3, mu=0.003, Pr=0.72), W3, dW3)
    B = cyl(16, 0.3, -1.0, 9)
    la, lb = cg.Mesh(A[0], order_tile=53), cg.Mesh(B[0], order_tile=29)
    tot = np.array(counts(la)) + np.array(counts(lb))
    pool = cg.Batch.pool(2, 3, *[int(x) for x in tot], precision=precision)
    sb = pool.admit(lb, B[1])
    pool.upload(sb, B[2], B[3])
    sa = pool.admit(la, A[1])
    pool.upload(sa, A[2], A[3])
    pool.cycle()
    pool.release(sb)
    pool.cycle()
    Wp, dWp = pool.download(sa)
    Wa, dWa = alone(A[0], A[1], A[2], A[3], 2, precision)
    assert np.array_equal(Wp, Wa) and np.array_equal(dWp, dWa)
    # 3-D: a batch of one tiled case against the same case in one tile
    bt = cg.Batch([cg.Mesh(m3, order_tile=41)], [S3[1]], precision=precision)
    b1 = cg.Batch([cg.Mesh(m3, order_tile=10**9)], [S3[1]], precision=precision)
    for b in (bt, b1):
        b.upload(0, W3, dW3)
        for _ in range(2):
            b.cycle()
    assert all(np.array_equal(x, y) for x, y in zip(bt.download(0), b1.download(0)))


def test_admission_is_bounded_by_capacity_and_reuses_ranges():
    cases = [cyl(32, 0.2 + 0.02 * k, 0.0, k) for k in range(4)]
    lm = [cg.Mesh(c[0]) for c in cases]
    one = np.array(counts(lm[0]))
    pool = cg.Batch.pool(2, 8, *[int(x) for x in 2 * one])     # room for two cases
    s0 = pool.admit(lm[0], cases[0][1])
    s1 = pool.admit(lm[1], cases[1][1])
    assert s0 is not None and s1 is not None
    assert pool.admit(lm[2], cases[2][1]) is None          # no cells left: waits
    off1 = pool.cell_off[s1]
    pool.release(s1)
    s2 = pool.admit(lm[2], cases[2][1])
    assert s2 is not None and pool.cell_off[s2] == off1     # first fit reuses the range
    pool.upload(s0, cases[0][2], cases[0][3])
    pool.upload(s2, cases[2][2], cases[2][3])
    res = pool.solve(max_cycles=3, tol=0.0, check_every=1)[0]
    assert [r["cycles"] for r in res if r["cycles"]] == [3, 3]
    W2, _ = pool.download(s2)
    Wa, _ = alone(cases[2][0], cases[2][1], cases[2][2], cases[2][3], 3)
    assert np.array_equal(W2, Wa)


def test_pool_graph_replays_after_admission():
    import torch
    A, B = cyl(32, 0.2, 1.0, 5), cyl(16, 0.3, -2.0, 6)
    la, lb = cg.Mesh(A[0]), cg.Mesh(B[0])
    tot = np.array(counts(la)) + np.array(counts(lb))
    pool = cg.Batch.pool(2, 4, *[int(x) for x in tot])
    sa = pool.admit(la, A[1])
    pool.upload(sa, A[2], A[3])
    pool.graph_create(2)
    pool.graph_launch()
    sb = pool.admit(lb, B[1])               # drops the graph: capture again
    pool.upload(sb, B[2], B[3])
    pool.graph_create(2)
    hist = torch.zeros(2 * pool.n_case, dtype=torch.float64, device="cuda")
    pool.graph_launch(hist)
    torch.cuda.synchronize()
    Wa, _ = alone(A[0], A[1], A[2], A[3], 4)
    Wb, _ = alone(B[0], B[1], B[2], B[3], 2)
    assert np.array_equal(pool.download(sa)[0], Wa)
    assert np.array_equal(pool.download(sb)[0], Wb)


def test_pool_case_matches_oracle():
    m = I.sphere_mesh(6, 12, 7, 2, 3)
    w = I.free_stream(3, 0.3, 5.0)
    kw = dict(W_inf=w, mu=0.003, Pr=0.72)
    W, dW = I.smooth_state(m, w, seed=9, amp=0.03)
    lm = cg.Mesh(m)
    n = np.array(counts(lm))
    pool = cg.Batch.pool(3, 2, *[int(x) for x in 2 * n])
    filler = pool.admit(lm, cg.Params(**kw))            # occupies the first ranges
    s = pool.admit(lm, cg.Params(**kw))
    pool.upload(filler, W, dW)
    pool.upload(s, W, dW)
    pool.release(filler)
    so = oracle.Solver(oracle.Mesh(m), oracle.Params(**kw))
    Wo, dWo = W.copy(), dW.copy()
    for _ in range(2):
        so.cycle(Wo, dWo)
        pool.cycle()
    Wg, dWg = pool.download(s)
    assert np.abs(Wg - Wo).max() <= 1e-11 * np.abs(Wo).max()
    assert np.abs(dWg - dWo).max() <= 1e-10 * np.abs(dWo).max()


def test_large_capacity_pool_equals_alone():
    """A 3-D pool whose cell capacity times the 45 packed operator entries
    per cell passes 2^31 (structure-of-arrays offsets need 64 bits): a case
    in it equals the same case alone, bitwise."""
    m = I.cubed_sphere_mesh(4, 8, 3, 2)
    w = I.free_stream(3, 0.3, 3.0)
    p = cg.Params(W_inf=w, mu=0.003, Pr=0.72)
    W, dW = I.smooth_state(m, w, seed=12, amp=0.02)
    lm = cg.Mesh(m)
    nc, nf, ng, nb = counts(lm)
    cap_cells = 50_000_000
    pool = cg.Batch.pool(3, 2, cap_cells, 2 * nf, 2 * ng, 2 * nb)
    s = pool.admit(lm, p)
    pool.upload(s, W, dW)
    for _ in range(3):
        pool.cycle()
    Wp, dWp = pool.download(s)
    Wa, dWa = alone(m, p, W, dW, 3)
    assert np.array_equal(Wp, Wa) and np.array_equal(dWp, dWa)
    del pool
