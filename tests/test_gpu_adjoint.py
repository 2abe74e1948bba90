"""The hand-written adjoint (dis_flow_backward) against the oracle's autograd
gradient and against central finite differences of the GPU forward, in
float64 (DIS_FLAG_IO_F64), plus the float32 interface, the autograd Function
and the error paths.

Loss throughout: mean end-point error of the flow against the generated
ground truth (differentiable differential-flow workload: pairs of 512x256
from the smooth-bump generator, 32x32 crops for the finite differences).
Every GPU test prints its case before it touches the device.
"""
import sys

import numpy as np
import pytest
import torch

from dis_cases import oracle_params, pair
from oracle import dis_oracle as O
from paper_1603_03590_amd import DIS, DisError, dis_flow, params, _lib

pytestmark = pytest.mark.gpu

F64 = 0x10
KEEP = 0x1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def crop(k, w=32, h=32, seed0=2000):
    """Crop of pair k of the 8-pair 512x256 bump batch, top-left (64k, 64)."""
    pr = pair("bump", 512, 256, 16.0, seed0 + k)
    x0, y0 = 64 * k, 64
    return (np.ascontiguousarray(pr.I0[y0:y0 + h, x0:x0 + w]), np.ascontiguousarray(pr.I1[y0:y0 + h, x0:x0 + w]),
            np.ascontiguousarray(pr.flow[:, y0:y0 + h, x0:x0 + w]))


def epe_loss(flow, gt):
    return torch.sqrt(((flow - gt) ** 2).sum(0)).mean()


def oracle_grad(I0, I1, gt, p):
    a = torch.from_numpy(I0).to(torch.float64).requires_grad_(True)
    b = torch.from_numpy(I1).to(torch.float64).requires_grad_(True)
    L = epe_loss(O.dis_flow(a, b, oracle_params(p)), torch.from_numpy(gt).to(torch.float64))
    g0, g1 = torch.autograd.grad(L, (a, b))
    return float(L.detach()), g0.numpy(), g1.numpy()


def gpu_grad(I0, I1, gt, p, d=None):
    """Loss and gradients through the autograd Function on the GPU."""
    h, w = I0.shape
    own = d is None
    if own:
        d = DIS(p, w, h)
    dt = d.dtype
    a = torch.from_numpy(I0).to(dt).cuda().requires_grad_(True)
    b = torch.from_numpy(I1).to(dt).cuda().requires_grad_(True)
    L = epe_loss(dis_flow(a, b, d), torch.from_numpy(gt).to(dt).cuda())
    L.backward()
    torch.cuda.synchronize()
    out = float(L.detach()), a.grad.double().cpu().numpy(), b.grad.double().cpu().numpy()
    if own:
        d.close()
    return out


def rel_err(g, ref):
    return float(np.abs(g - ref).max() / max(np.abs(ref).max(), 1e-300))


VARIANTS = [
    # name, crop (k, w, h), preset, overrides
    ("c5_crop0", (0, 32, 32), 105, {}),
    ("c5_crop3", (3, 32, 32), 105, {}),
    ("c5_crop5_ragged_45x37", (5, 45, 37), 105, {}),
    ("norefine", (1, 32, 32), 105, dict(refine=0)),
    ("raw_residual_pixel_centre", (2, 40, 32), 105, dict(flags=0x8 | 0x4)),
    ("finest_scale_1", (4, 48, 40), 105, dict(finest_scale=1, coarsest_scale=2)),
    ("vi7_phases_split", (6, 32, 32), 105, dict(var_inner=7)),
    ("vo0_no_fixed_point", (7, 32, 32), 105, dict(var_outer=0)),
    ("vo_auto_s_plus_1", (0, 40, 40), 105, dict(var_outer=-1)),
    ("ps4_ov0", (1, 24, 24), 105, dict(patch_size=4, overlap=0.0, gn_iters=8)),
    ("ps12_ov075_single_level", (2, 32, 32), 105, dict(patch_size=12, overlap=0.75, coarsest_scale=0, gn_iters=20)),
    ("gn0_init_only", (3, 32, 32), 105, dict(gn_iters=0)),
    # one scale from a zero start to motions of about 5 px: the reverse
    # search's iterates leave the patch's LDS window (which then spans the
    # start and the end) part of the way, so both its sampling paths run
    ("ps8_single_level_5px", (1, 40, 40), 105, dict(coarsest_scale=0)),
    ("ps6_window", (5, 36, 36), 105, dict(patch_size=6)),
]


@pytest.mark.parametrize("name,cr,preset,over", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_adjoint_matches_oracle_autograd(name, cr, preset, over):
    say(f"[adjoint] case {name} crop {cr}")
    I0, I1, gt = crop(*cr)
    over = dict(over)
    over["flags"] = over.get("flags", 0) | F64 | KEEP
    p = params(preset, **over)
    L_ref, r0, r1 = oracle_grad(I0, I1, gt, p)
    L, g0, g1 = gpu_grad(I0, I1, gt, p)
    e0, e1 = rel_err(g0, r0), rel_err(g1, r1)
    say(f"[adjoint] {name}: loss {L:.12g} (oracle {L_ref:.12g}), rel max err dI0 {e0:.2e} dI1 {e1:.2e}")
    assert abs(L - L_ref) <= 1e-9 * abs(L_ref)
    assert e0 <= 1e-7 and e1 <= 1e-7


def test_adjoint_full_size_512x256_matches_oracle():
    """One whole pair of the 8-pair batch at its real size and parameters."""
    say("[adjoint] case c5_full_512x256 seed 2000")
    pr = pair("bump", 512, 256, 16.0, 2000)
    p = params(105, flags=F64 | KEEP)
    L_ref, r0, r1 = oracle_grad(pr.I0, pr.I1, pr.flow, p)
    L, g0, g1 = gpu_grad(pr.I0, pr.I1, pr.flow, p)
    e0, e1 = rel_err(g0, r0), rel_err(g1, r1)
    say(f"[adjoint] c5_full: loss {L:.12g} (oracle {L_ref:.12g}), rel max err {e0:.2e} {e1:.2e}")
    assert abs(L - L_ref) <= 1e-9 * abs(L_ref)
    assert e0 <= 1e-6 and e1 <= 1e-6


@pytest.mark.parametrize("k", [0, 2, 4, 6])
def test_adjoint_matches_finite_differences(k):
    """Directional derivatives <dL/dI, v> (v dense Gaussian) against central
    differences of the GPU forward in float64.  The loss is only piecewise
    smooth (bilinear cells, the 1/max(1,|d|) weights, the reset test), so the
    step must be small enough that the perturbed path crosses no kink:
    1e-9 on frames in [0, 1] (the oracle's own differences agree with its
    autograd gradient to a few 1e-5 there, and drift away for 1e-7 and up)."""
    say(f"[adjoint-fd] crop {k}")
    I0, I1, gt = crop(k)
    p = params(105, flags=F64 | KEEP)
    d = DIS(p, 32, 32)
    try:
        _, g0, g1 = gpu_grad(I0, I1, gt, p, d)
        gt_t = torch.from_numpy(gt).double().cuda()
        rng = np.random.default_rng(100 + k)

        def loss(a, b):
            with torch.no_grad():
                f = d.flow(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
                return float(epe_loss(f, gt_t))

        a0, a1 = I0.astype(np.float64), I1.astype(np.float64)
        eps = 1e-9
        for trial in range(3):
            v0 = rng.standard_normal(a0.shape)
            v1 = rng.standard_normal(a1.shape)
            fd = (loss(a0 + eps * v0, a1 + eps * v1) - loss(a0 - eps * v0, a1 - eps * v1)) / (2 * eps)
            an = float((g0 * v0).sum() + (g1 * v1).sum())
            say(f"[adjoint-fd] crop {k} dir {trial}: fd {fd:.10e} adjoint {an:.10e}")
            assert abs(fd - an) <= 2e-4 * max(abs(fd), abs(an)) + 1e-6
    finally:
        d.close()


def test_adjoint_float32_interface_close_to_float64():
    say("[adjoint] case f32 vs f64 crop 1")
    I0, I1, gt = crop(1)
    _, d0, d1 = gpu_grad(I0, I1, gt, params(105, flags=F64 | KEEP))
    _, s0, s1 = gpu_grad(I0, I1, gt, params(105, flags=KEEP))
    e0, e1 = rel_err(s0, d0), rel_err(s1, d1)
    say(f"[adjoint] f32 vs f64: {e0:.2e} {e1:.2e}")
    assert e0 <= 1e-4 and e1 <= 1e-4


def test_backward_repeat_and_graph_agree_with_eager():
    """Replays of the backward graph (several calls, gradient buffers moved)
    and the launch-by-launch path give the same gradients."""
    say("[adjoint] case replay / eager crop 2")
    I0, I1, gt = crop(2)
    ref = gpu_grad(I0, I1, gt, params(105, flags=F64 | KEEP | 0x2))
    d = DIS(params(105, flags=F64 | KEEP), 32, 32)
    try:
        for _ in range(3):
            got = gpu_grad(I0, I1, gt, None, d)
            assert rel_err(got[1], ref[1]) <= 1e-12 and rel_err(got[2], ref[2]) <= 1e-12
    finally:
        d.close()


@pytest.mark.parametrize("name,cr,over", [
    ("c5_crop6", (6, 32, 32), {}),
    ("ragged_45x37", (5, 45, 37), {}),
    ("vi7_two_launches_per_step", (2, 40, 32), dict(var_inner=7)),
    ("vo_auto_sf1", (4, 48, 40), dict(var_outer=-1, finest_scale=1, coarsest_scale=2)),
    # finest scale wide enough for 16x16 reverse cores (two launches per step)
    ("cores16_256x128", (0, 256, 128), {}),
])
def test_tiled_reverse_sweeps_match_reference_form(name, cr, over):
    """The tiled reverse of each fixed-point step against one launch per
    reverse half sweep (launch mode bit 2) and against a handle whose forward
    runs the coarser scales as single workgroups (bits 1 and 4; the finest
    scale, whose tape the forward keeps, runs tiled, and the adjoint
    recomputes the coarser ones tiled), and all against the oracle."""
    say(f"[adjoint] case tiled vs reference {name}")
    I0, I1, gt = crop(*cr)
    h, w = I0.shape
    p = params(105, flags=F64 | KEEP, **over)
    grads = []
    for mode in (1, 1 | 4, 1 | 2 | 16):
        d = DIS(p, w, h)
        try:
            d.set_tunables(None, 7, mode)
            grads.append(gpu_grad(I0, I1, gt, p, d))
        finally:
            d.close()
    _, r0, r1 = oracle_grad(I0, I1, gt, p)
    (_, t0, t1), (_, f0, f1), (_, s0, s1) = grads
    say(f"[adjoint] {name}: tiled vs reference {rel_err(t0, f0):.2e} {rel_err(t1, f1):.2e}, "
        f"single-workgroup {rel_err(s0, t0):.2e}, tiled vs oracle {rel_err(t0, r0):.2e}")
    assert rel_err(t0, f0) <= 1e-11 and rel_err(t1, f1) <= 1e-11
    assert rel_err(s0, t0) <= 1e-11 and rel_err(s1, t1) <= 1e-11
    assert rel_err(t0, r0) <= 1e-7 and rel_err(t1, r1) <= 1e-7


def test_backward_after_other_size_forward():
    """One handle, two sizes: each backward differentiates its own forward."""
    say("[adjoint] case two sizes on one handle")
    p = params(105, flags=F64 | KEEP)
    d = DIS(p, 48, 40)
    try:
        for k, (w, h) in ((3, (48, 40)), (4, (32, 32)), (3, (48, 40))):
            I0, I1, gt = crop(k, w, h)
            _, g0, g1 = gpu_grad(I0, I1, gt, p, d)
            _, r0, r1 = oracle_grad(I0, I1, gt, p)
            assert rel_err(g0, r0) <= 1e-7 and rel_err(g1, r1) <= 1e-7
    finally:
        d.close()


def test_backward_errors():
    say("[adjoint] case error paths")
    I0, I1, gt = crop(0)
    g = torch.zeros((2, 32, 32), dtype=torch.float64, device="cuda")
    # handle without KEEP_FOR_BACKWARD
    d = DIS(params(105, flags=F64), 32, 32)
    try:
        d.flow(torch.from_numpy(I0).double().cuda(), torch.from_numpy(I1).double().cuda())
        with pytest.raises(DisError) as e:
            d.backward(g)
        assert e.value.code == _lib.DIS_ESTATE
    finally:
        d.close()
    d = DIS(params(105, flags=F64 | KEEP), 32, 32, max_batch=2)
    try:
        # no forward yet
        with pytest.raises(DisError) as e:
            d.backward(g)
        assert e.value.code == _lib.DIS_ESTATE
        a = torch.from_numpy(I0).double().cuda()
        b = torch.from_numpy(I1).double().cuda()
        # a batched call replaces the plain forward
        d.flow(a, b)
        d.flow_batched([a, a], [b, b])
        with pytest.raises(DisError) as e:
            d.backward(g)
        assert e.value.code == _lib.DIS_ESTATE
        # the adjoint covers the two-dimensional L2 search only
        for extra in (dict(norm=1), dict(flags=F64 | KEEP | 0x20)):
            over = dict(flags=F64 | KEEP)
            over.update(extra)
            dn = DIS(params(105, **over), 32, 32)
            try:
                dn.flow(a, b)
                with pytest.raises(DisError) as e:
                    dn.backward(g)
                assert e.value.code == _lib.DIS_EINVAL
            finally:
                dn.close()
        # more Gauss-Newton iterations than the reverse search keeps in LDS
        # (134 for 8x8 patches); the limit itself runs
        for iters, ok in ((135, False), (134, True)):
            dn = DIS(params(105, flags=F64 | KEEP, gn_iters=iters), 32, 32)
            try:
                dn.flow(a, b)
                if ok:
                    dn.backward(g)
                else:
                    with pytest.raises(DisError) as e:
                        dn.backward(g)
                    assert e.value.code == _lib.DIS_EINVAL and "at most 134" in str(e.value)
            finally:
                dn.close()
        # the autograd Function refuses a stale forward
        a2 = a.clone().requires_grad_(True)
        f = dis_flow(a2, b, d)
        d.flow(a, b)
        with pytest.raises(RuntimeError):
            f.sum().backward()
    finally:
        d.close()
    torch.cuda.synchronize()


def test_forward_kept_for_backward_is_the_plain_forward():
    """A forward kept for the adjoint (which records the finest scale's SOR
    tape, weight sums, warped frame and linearisation on the way, and runs
    that scale tiled) returns the plain forward's flow bit for bit, in every
    launch mode."""
    say("[adjoint] case kept forward vs plain forward, 512x256")
    pr = pair("bump", 512, 256, 16.0, 2000)
    a = torch.from_numpy(pr.I0).to(torch.float64).cuda()
    b = torch.from_numpy(pr.I1).to(torch.float64).cuda()
    for mode in (1, 3, 9, 0, 1 | 2 | 16):
        outs = []
        for flags in (F64, F64 | KEEP):
            d = DIS(params(105, flags=flags), 512, 256)
            try:
                d.set_tunables(None, 7, mode)
                outs.append(d.flow(a, b).cpu().numpy())
                torch.cuda.synchronize()
            finally:
                d.close()
        assert np.array_equal(outs[0], outs[1]), mode
