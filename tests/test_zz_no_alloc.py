"""The residual entry point for callers that cannot allocate
(cgks_residual_high_noalloc): its work arrays live in the library's fixed
device scratch, and it must return bitwise the transferred residual R1 of
cgks_residual(CGKS_RESIDUAL_HIGH) on the same state, call after call, also
when a later call covers a smaller batch than an earlier one."""
import numpy as np
import pytest

import paper_2109_09965_amd as cg
import paper_2109_09965_amd.inputs as I


def _batch(mesh, precision, seed, mach=0.3, mu=0.01):
    d = mesh["dim"]
    Winf = I.free_stream(d, mach, 7.0)
    W, dW = I.smooth_state(mesh, Winf, seed=seed, amp=0.04)
    b = cg.Batch([cg.Mesh(mesh)], [cg.Params(W_inf=Winf, mu=mu, Pr=0.72)], precision=precision)
    b.upload(0, W, dW)
    return b


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [cg.FP64, cg.MIXED32, cg.MIXED32_R64])
def test_noalloc_residual_equals_arena_residual(precision):
    import torch
    cases = [
        lambda: I.cubed_sphere_mesh(6, 10, 5, 3, wall=I.BC_NOSLIP_ADIABATIC),   # 2,160 cells
        lambda: I.box3d_mesh((3, 3, 4), layer_types=["tet", "prism", "hex", "pyr"], perturb=0.2, seed=2),
        lambda: I.cylinder_mesh(32, 16, wall=I.BC_SLIP_WALL),                     # 1,024 cells
        lambda: I.box2d_mesh(6, periodic=False, perturb=0.2, seed=3),
    ]
    for k, mk in enumerate(cases):
        mesh = mk()
        b = _batch(mesh, precision, seed=k + 1)
        print(f"noalloc: precision {precision} case {k}: {mesh['n_cell']} cells", flush=True)
        ref = b.residual(cg.RESIDUAL_HIGH).cpu().numpy()
        out = torch.full((b.nv * b.NC,), float("nan"), dtype=torch.float64, device=b.arena.device)
        got = b.residual_high_noalloc(out).cpu().numpy()
        torch.cuda.synchronize()
        assert np.isfinite(ref).all()
        np.testing.assert_array_equal(got, ref)
        # a second call on the same batch gives the same again
        got2 = b.residual_high_noalloc().cpu().numpy()
        np.testing.assert_array_equal(got2, ref)


@pytest.mark.gpu
def test_noalloc_rejects_batches_beyond_the_scratch():
    """A batch whose residual pass needs more than the fixed scratch is
    refused with CGKS_ENOMEM before anything is launched."""
    mesh = I.cubed_sphere_mesh(16, 30)          # 61,440 cells: about 80 MiB of FP64 records and face sums
    b = _batch(mesh, cg.FP64, seed=9, mach=0.25)
    with pytest.raises(cg.CgksError) as e:
        b.residual_high_noalloc()
    assert e.value.status == cg.ENOMEM
    # the batch itself is untouched and still works through the arena
    assert np.isfinite(b.residual(cg.RESIDUAL_HIGH).cpu().numpy()).all()
