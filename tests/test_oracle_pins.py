"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these retype the oracle's formulas: each checks a closed form, an
invariant, a special case solved by another route, or a constant the paper
prints (tests/golden/paper_constants.json).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

from oracle import dis_oracle as O
from oracle import search_checks as SC

F64 = torch.float64
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def analytic_texture(h, w, shift=(0.0, 0.0), seed=0, min_period=20.0, n=12):
    """0.5 + sum of sinusoids, evaluated exactly at (x - tx, y - ty)."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    xx = xx - shift[0]
    yy = yy - shift[1]
    out = np.full((h, w), 0.5)
    for _ in range(n):
        per = rng.uniform(min_period, 3 * min_period)
        ang = rng.uniform(0, 2 * math.pi)
        ph = rng.uniform(0, 2 * math.pi)
        fx, fy = math.cos(ang) / per, math.sin(ang) / per
        out += (0.4 / n) * np.sin(2 * math.pi * (fx * xx + fy * yy) + ph)
    return torch.from_numpy(out)


def params(**kw):
    base = dict(patch_size=8, overlap=0.5, coarsest_scale=3, finest_scale=0, gn_iters=16,
                var_outer=3, var_inner=5, refine=True)
    base.update(kw)
    return O.OracleParams(**base)


# ------------------------------------------------------------------ P1 -------
@pytest.mark.parametrize("refine", [False, True])
def test_p1_identical_frames_give_exactly_zero_flow(refine):
    I = analytic_texture(96, 128, seed=1)
    for sf in (0, 2):
        U = O.dis_flow(I, I.clone(), params(refine=refine, finest_scale=sf))
        assert torch.count_nonzero(U) == 0


# ------------------------------------------------------------------ P2 -------
@pytest.mark.parametrize("t", [(5.3, -3.7), (-11.6, 7.25), (0.4, 0.2)])
@pytest.mark.parametrize("refine", [False, True])
def test_p2_global_translation(t, refine):
    h, w = 128, 160
    I0 = analytic_texture(h, w, seed=2)
    I1 = analytic_texture(h, w, shift=t, seed=2)     # I1(x + t) = I0(x)
    U = O.dis_flow(I0, I1, params(refine=refine, coarsest_scale=3, gn_iters=16))
    m = int(abs(t[0]) + abs(t[1])) + 10
    err = torch.sqrt((U[0] - t[0]) ** 2 + (U[1] - t[1]) ** 2)[m:h - m, m:w - m]
    assert err.mean() < 0.05, float(err.mean())


# ------------------------------------------------------------------ P3 -------
@pytest.mark.parametrize("rot_deg,scale", [(1.0, 1.0), (-1.0, 0.99), (0.0, 1.02)])
def test_p3_small_affine_motion(rot_deg, scale):
    """Rigid patches cannot follow a rotation exactly: the model error grows
    with the flow gradient times the patch size (about 5% of the largest
    displacement here), so the warps stay within 1 degree / 2 percent."""
    h, w = 128, 160
    c = np.array([(w - 1) / 2, (h - 1) / 2])
    th = math.radians(rot_deg)
    A = scale * np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    Ainv = np.linalg.inv(A)
    rng = np.random.default_rng(3)
    comps = [(rng.uniform(20, 60), rng.uniform(0, 2 * math.pi), rng.uniform(0, 2 * math.pi)) for _ in range(12)]

    def tex(x, y):
        out = np.full(x.shape, 0.5)
        for per, ang, ph in comps:
            out += (0.4 / 12) * np.sin(2 * math.pi * (math.cos(ang) * x + math.sin(ang) * y) / per + ph)
        return out

    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    I0 = tex(xx, yy)
    q = Ainv @ (np.stack([xx.ravel(), yy.ravel()]) - c[:, None]) + c[:, None]
    I1 = tex(q[0].reshape(h, w), q[1].reshape(h, w))   # I1(A(x-c)+c) = I0(x)
    gt = (A - np.eye(2)) @ (np.stack([xx.ravel(), yy.ravel()]) - c[:, None])
    U = O.dis_flow(torch.from_numpy(I0), torch.from_numpy(I1), params(coarsest_scale=3))
    err = np.sqrt((U[0].numpy().ravel() - gt[0]) ** 2 + (U[1].numpy().ravel() - gt[1]) ** 2).reshape(h, w)
    m = 12
    assert err[m:h - m, m:w - m].mean() < 0.1, err[m:h - m, m:w - m].mean()


# ------------------------------------------------------------------ P4 -------
def test_p4_bilinear_image_gn_converges_to_exact_translation():
    """On a bilinear image Sobel/8 is the exact derivative and bilinear
    interpolation is exact, so u = t is an exact fixed point.  With the
    template gradient left uncentred (R9) the step's contraction factor is
    g_mean^T (sum g g^T / n)^-1 g_mean, which vanishes when the patch is
    centred on the saddle of J0 = c (x - xs)(y - ys): convergence is then
    essentially exact within a few iterations."""
    h, w = 48, 56
    c = 0.8
    t = (0.7, -0.4)
    x0, y0 = 20, 18
    xs, ys = x0 + 3.5, y0 + 3.5
    yy, xx = torch.meshgrid(torch.arange(h, dtype=F64), torch.arange(w, dtype=F64), indexing="ij")
    J0 = c * (xx - xs) * (yy - ys) + 100.0
    J1 = c * (xx - t[0] - xs) * (yy - t[1] - ys) + 100.0
    Gx, Gy = O.sobel8(J0)
    assert torch.allclose(Gx[1:-1, 1:-1], (c * (yy - ys))[1:-1, 1:-1], atol=1e-12)
    assert torch.allclose(Gy[1:-1, 1:-1], (c * (xx - xs))[1:-1, 1:-1], atol=1e-12)
    tt = torch.tensor([t], dtype=F64)
    res = O.inverse_search(J0, Gx, Gy, J1, torch.tensor([x0]), torch.tensor([y0]),
                           torch.zeros(1, 2, dtype=F64), params(gn_iters=8, patch_size=8))
    assert (res.u - tt).abs().max() < 1e-9
    # off the saddle the same fixed point is reached, linearly
    res = O.inverse_search(J0, Gx, Gy, J1, torch.tensor([x0 + 3]), torch.tensor([y0 - 2]),
                           torch.zeros(1, 2, dtype=F64), params(gn_iters=200, patch_size=8))
    assert (res.u - tt).abs().max() < 1e-9


# ------------------------------------------------------------------ P5 -------
def test_p5_hessian_symmetric_psd_and_independent():
    rng = np.random.default_rng(5)
    J = ndi.gaussian_filter(rng.standard_normal((40, 40)), 1.5) * 60 + 128
    Jt = torch.from_numpy(J)
    Gx, Gy = O.sobel8(Jt)
    x0, y0, _, _ = O.patch_grid(40, 40, params(patch_size=8, overlap=0.5))
    res = O.inverse_search(Jt, Gx, Gy, Jt, x0, y0, torch.zeros(len(x0), 2, dtype=F64), params(gn_iters=1))
    H = res.hessian
    assert torch.equal(H, H.transpose(1, 2))
    ev = torch.linalg.eigvalsh(H)
    assert (ev > 0).all()
    # independent gradient: scipy's Sobel with replicated border, divided by 8
    gx = ndi.sobel(J, axis=1, mode="nearest") / 8.0
    gy = ndi.sobel(J, axis=0, mode="nearest") / 8.0
    for i in range(len(x0)):
        X, Y = int(x0[i]), int(y0[i])
        px = gx[Y:Y + 8, X:X + 8].ravel()
        py = gy[Y:Y + 8, X:X + 8].ravel()
        Hi = np.array([[px @ px, px @ py], [px @ py, py @ py]])
        assert np.allclose(H[i].numpy(), Hi, rtol=1e-12, atol=1e-9)


def test_p5_hessian_of_a_ramp():
    a = 2.5
    J = torch.arange(30, dtype=F64)[None, :].repeat(30, 1) * a
    Gx, Gy = O.sobel8(J)
    res = O.inverse_search(J, Gx, Gy, J, torch.tensor([10]), torch.tensor([10]), torch.zeros(1, 2, dtype=F64),
                           params(gn_iters=0))
    assert torch.allclose(res.hessian[0], torch.tensor([[64 * a * a, 0.0], [0.0, 0.0]], dtype=F64))


# ------------------------------------------------------------------ P6 -------
@pytest.mark.parametrize("ps", [8, 12])
@pytest.mark.parametrize("noise,tol", [(0.0, 1e-2), (0.5, 5e-2)])
def test_p6_inverse_search_agrees_with_forward_additive_and_brute_force(ps, noise, tol):
    t = (0.37, -0.62)
    n = ps + 16
    J0 = 255 * analytic_texture(n, n, seed=6, min_period=10.0)
    J1 = 255 * analytic_texture(n, n, shift=t, seed=6, min_period=10.0)
    if noise:
        J1 = J1 + torch.from_numpy(np.random.default_rng(7).normal(0, noise, J1.shape))
    x0 = y0 = 8
    Gx, Gy = O.sobel8(J0)
    ic = O.inverse_search(J0, Gx, Gy, J1, torch.tensor([x0]), torch.tensor([y0]),
                          torch.zeros(1, 2, dtype=F64), params(gn_iters=60, patch_size=ps)).u[0]
    fa = SC.forward_additive_lk(J0, J1, x0, y0, ps, [0.0, 0.0], iters=60)
    bf = SC.brute_force(J0, J1, x0, y0, ps, t, radius=1.0)
    assert (ic - bf).norm() < tol, (ic, bf)
    assert (fa - bf).norm() < 0.01, (fa, bf)
    assert (ic - fa).norm() < tol


# ------------------------------------------------------------------ P7 -------
def test_p7_constant_offset_of_second_frame_does_not_change_flow():
    from paper_1603_03590_amd import synth
    pr = synth.smooth_bump_pair(128, 96, 6.0, 11)
    I0 = torch.from_numpy(pr.I0).to(F64)
    I1 = torch.from_numpy(pr.I1).to(F64)
    for sf in (0, 1):
        p = params(refine=False, coarsest_scale=3, finest_scale=sf)
        U = O.dis_flow(I0, I1, p)
        U2 = O.dis_flow(I0, I1 + 0.137, p)
        assert (U - U2).abs().max() < 1e-12


# ------------------------------------------------------------------ P8 -------
def test_p8_reset_of_a_diverging_patch():
    rng = np.random.default_rng(8)
    h, w = 32, 32
    # a nearly flat template (tiny H) against a strongly textured second frame
    J0 = torch.from_numpy(100.0 + 0.02 * rng.standard_normal((h, w)))
    J1 = torch.from_numpy(ndi.gaussian_filter(rng.standard_normal((h, w)), 1.0) * 80 + 100)
    Gx, Gy = O.sobel8(J0)
    uinit = torch.tensor([[0.3, -0.2], [1.0, 2.0]], dtype=F64)
    res = O.inverse_search(J0, Gx, Gy, J1, torch.tensor([8, 16]), torch.tensor([8, 16]), uinit, params(gn_iters=4))
    moved = (res.u_search - uinit).norm(dim=1)
    assert (moved > 8).all()                       # the search ran away ...
    assert res.reset.all()
    assert torch.equal(res.u, uinit)               # ... and was reset to its start


def test_p8_no_reset_when_within_patch_size():
    I0 = analytic_texture(64, 64, seed=9, min_period=8.0, n=24)
    I1 = analytic_texture(64, 64, shift=(1.5, -0.5), seed=9, min_period=8.0, n=24)
    J0, J1 = 255 * I0, 255 * I1
    Gx, Gy = O.sobel8(J0)
    x0, y0, _, _ = O.patch_grid(64, 64, params())
    res = O.inverse_search(J0, Gx, Gy, J1, x0, y0, torch.zeros(len(x0), 2, dtype=F64), params())
    assert not res.reset.any()
    assert torch.equal(res.u, res.u_search)
    # short-period texture: bilinear interpolation error keeps this at ~0.05 px
    assert (res.u - torch.tensor([1.5, -0.5], dtype=F64)).norm(dim=1).median() < 0.1


# ------------------------------------------------------------------ P9 -------
def test_p9_densification_is_a_normalised_average():
    rng = np.random.default_rng(10)
    w, h = 37, 29
    p = params(patch_size=8, overlap=0.5)
    x0, y0, nx, ny = O.patch_grid(w, h, p)
    n = len(x0)
    d = torch.from_numpy(rng.normal(0, 5, (n, 64)))
    c = torch.tensor([1.25, -3.5], dtype=F64)
    U, Z = O.densify(w, h, x0, y0, c.repeat(n, 1), d, p)
    assert (U[0] - c[0]).abs().max() < 1e-13 and (U[1] - c[1]).abs().max() < 1e-13
    u = torch.from_numpy(rng.normal(0, 3, (n, 2)))
    U, Z = O.densify(w, h, x0, y0, u, d, p)
    # convex combination of the covering patches
    lo = torch.full((2, h, w), float("inf"), dtype=F64)
    hi = torch.full((2, h, w), -float("inf"), dtype=F64)
    for i in range(n):
        X, Y = int(x0[i]), int(y0[i])
        for k in range(2):
            lo[k, Y:Y + 8, X:X + 8] = torch.minimum(lo[k, Y:Y + 8, X:X + 8], u[i, k])
            hi[k, Y:Y + 8, X:X + 8] = torch.maximum(hi[k, Y:Y + 8, X:X + 8], u[i, k])
    assert (U >= lo - 1e-12).all() and (U <= hi + 1e-12).all()
    # the top-left pixel is covered by patch 0 alone
    assert torch.allclose(U[:, 0, 0], u[0], atol=0, rtol=1e-15)
    # the weight of a residual below 1 is 1, of |d| > 1 is 1/|d|: check one pixel by hand
    y, x = 5, 6
    cov = [i for i in range(n) if x0[i] <= x < x0[i] + 8 and y0[i] <= y < y0[i] + 8]
    wts = [1.0 / max(1.0, abs(float(d[i, (y - y0[i]) * 8 + (x - x0[i])]))) for i in cov]
    ref = sum(wt * float(u[i, 0]) for wt, i in zip(wts, cov)) / sum(wts)
    assert abs(float(U[0, y, x]) - ref) < 1e-12


# ------------------------------------------------------------------ P10 ------
@pytest.mark.parametrize("w,h,ps,ov", [(128, 54, 8, 0.4), (37, 29, 8, 0.3), (64, 48, 12, 0.75), (20, 9, 8, 0.0)])
def test_p10_grid_covers_every_pixel(w, h, ps, ov):
    p = params(patch_size=ps, overlap=ov)
    st = O.grid_stride(p)
    x0, y0, nx, ny = O.patch_grid(w, h, p)
    assert len(x0) == (math.ceil((w - ps) / st) + 1) * (math.ceil((h - ps) / st) + 1)
    cov = torch.zeros(h, w, dtype=torch.long)
    for X, Y in zip(x0.tolist(), y0.tolist()):
        assert 0 <= X <= w - ps and 0 <= Y <= h - ps
        cov[Y:Y + ps, X:X + ps] += 1
    assert (cov > 0).all()


def test_p10_paper_patch_count_at_scale_3():
    g = json.load(open(GOLDEN))["patch_count_scale3_sintel"]
    w, h = g["level_size"]
    p = params(patch_size=g["patch_size"], overlap=g["overlap"], grid="overhang")
    x0, _, _, _ = O.patch_grid(w, h, p)
    assert len(x0) == g["value"]
    assert O.level_sizes(1024, 436, 3)[-1] == (w, h)


# ------------------------------------------------------------------ P11 ------
def test_p11_coarsest_scale_rule_matches_paper():
    g = json.load(open(GOLDEN))
    s = g["coarsest_scale_sintel"]
    for ps in s["patch_sizes"]:
        assert O.auto_coarsest_scale(s["width"], ps) == s["value"]
    k = g["coarsest_scale_kitti"]
    for w in k["widths"]:
        assert O.auto_coarsest_scale(w, k["patch_size"]) == k["value"]
    # the clamp keeps the coarsest level at least one patch tall
    assert O.coarsest_scale(1242, 375, params(coarsest_scale=-1)) == 5
    assert O.coarsest_scale(32, 32, params(coarsest_scale=3)) == 2


# ------------------------------------------------------------------ P12 ------
def _level_problem(seed=12, h=40, w=48):
    from paper_1603_03590_amd import synth
    pr = synth.smooth_bump_pair(w, h, 3.0, seed)
    J0 = 255 * torch.from_numpy(pr.I0).to(F64)
    J1 = 255 * torch.from_numpy(pr.I1).to(F64)
    rng = np.random.default_rng(seed)
    U = torch.from_numpy(pr.flow + rng.normal(0, 0.3, pr.flow.shape))
    return J0, J1, U


def test_p12_refinement_energies_non_increasing():
    J0, J1, U = _level_problem()
    p = params(var_inner=5)
    log = []

    def trace(kind, k, t, sys, du, dv):
        log.append((kind, k, float(O.quadratic_energy(sys, U, du, dv)),
                    float(O.linearised_energy(t, U, du, dv, p))))

    O.refine(J0, J1, U, 6, p, trace)
    starts = {}
    prev_q = None
    for kind, k, q, e in log:
        if kind == "outer":
            starts[k] = e
            if k > 0:
                assert e <= starts[k - 1] * (1 + 1e-13)       # across fixed-point iterations
            prev_q = q
        else:
            assert q <= prev_q + 1e-9 * abs(prev_q)            # majoriser after each half sweep
            prev_q = q
            assert e <= starts[k] * (1 + 1e-13)                # robust energy below its start
    assert log[-1][3] < log[0][3]


# ------------------------------------------------------------------ P13 ------
def test_p13_many_sor_sweeps_solve_the_frozen_system():
    J0, J1, U = _level_problem(seed=13, h=14, w=17)
    p = params()
    t = O.refine_linearise(J0, J1, U)
    zero = torch.zeros_like(U[0])
    sys = O.sor_system(t, U, zero, zero, p)
    du, dv = O.sor_sweeps(sys, U, zero, zero, 2000, p.sor_omega)
    # assemble the normal equations of the quadratic independently
    h, w = U.shape[1:]
    n = h * w
    idx = lambda y, x: y * w + x
    rows, cols, vals = [], [], []
    rhs = np.zeros(2 * n)
    A11, A12, A22 = sys.A11.numpy(), sys.A12.numpy(), sys.A22.numpy()
    b1, b2, ws = sys.b1.numpy(), sys.b2.numpy(), sys.ws.numpy()
    Un, Vn = U[0].numpy(), U[1].numpy()
    diag = np.zeros(2 * n)
    for y in range(h):
        for x in range(w):
            i = idx(y, x)
            rows += [i, n + i]
            cols += [n + i, i]
            vals += [A12[y, x], A12[y, x]]
            diag[i] += A11[y, x]
            diag[n + i] += A22[y, x]
            rhs[i] -= b1[y, x]
            rhs[n + i] -= b2[y, x]
            for (yy, xx) in ((y, x + 1), (y + 1, x)):
                if yy < h and xx < w:
                    j = idx(yy, xx)
                    wt = ws[y, x]
                    for off, F in ((0, Un), (n, Vn)):
                        diag[off + i] += wt
                        diag[off + j] += wt
                        rows += [off + i, off + j]
                        cols += [off + j, off + i]
                        vals += [-wt, -wt]
                        rhs[off + i] += wt * (F[yy, xx] - F[y, x])
                        rhs[off + j] += wt * (F[y, x] - F[yy, xx])
    M = sp.csr_matrix((vals + list(diag), (rows + list(range(2 * n)), cols + list(range(2 * n)))), shape=(2 * n, 2 * n))
    sol = spla.spsolve(M, rhs)
    assert np.allclose(du.numpy().ravel(), sol[:n], atol=1e-8)
    assert np.allclose(dv.numpy().ravel(), sol[n:], atol=1e-8)


# ------------------------------------------------------------------ P14 ------
def test_p14_without_smoothness_pixels_decouple():
    J0, J1, U = _level_problem(seed=14, h=12, w=15)
    p = params(alpha=0.0)
    t = O.refine_linearise(J0, J1, U)
    zero = torch.zeros_like(U[0])
    sys = O.sor_system(t, U, zero, zero, p)
    # some pixels are nearly rank one (A12^2 / (A11 A22) ~ 0.99): give them time
    du, dv = O.sor_sweeps(sys, U, zero, zero, 2000, p.sor_omega)
    det = sys.A11 * sys.A22 - sys.A12 ** 2
    ref_u = (-sys.b1 * sys.A22 + sys.b2 * sys.A12) / det
    ref_v = (-sys.b2 * sys.A11 + sys.b1 * sys.A12) / det
    assert torch.allclose(du, ref_u, atol=1e-9, rtol=1e-7)
    assert torch.allclose(dv, ref_v, atol=1e-9, rtol=1e-7)


def test_p14_constant_flow_without_temporal_terms_is_a_fixed_point():
    J0, J1, U = _level_problem(seed=15, h=12, w=15)
    U = torch.stack([torch.full_like(U[0], 1.75), torch.full_like(U[1], -0.5)])
    t = O.refine_linearise(J0, J1, U)
    t.Iz = torch.zeros_like(t.Iz)
    t.Ixz = torch.zeros_like(t.Ixz)
    t.Iyz = torch.zeros_like(t.Iyz)
    zero = torch.zeros_like(U[0])
    sys = O.sor_system(t, U, zero, zero, params())
    du, dv = O.sor_sweeps(sys, U, zero, zero, 5, 1.6)
    assert torch.count_nonzero(du) == 0 and torch.count_nonzero(dv) == 0


# ------------------------------------------------------------------ P15 ------
def test_p15_pyramid_box_means_by_hand():
    J = torch.tensor([[1., 2., 3., 4., 9.],
                      [5., 6., 7., 8., 9.],
                      [9., 10., 11., 12., 9.],
                      [13., 14., 15., 16., 9.],
                      [7., 7., 7., 7., 7.]], dtype=F64)
    L = O.build_pyramid(J, 2)
    assert torch.equal(L[1], torch.tensor([[3.5, 5.5], [11.5, 13.5]], dtype=F64))
    assert torch.equal(L[2], torch.tensor([[8.5]], dtype=F64))
    assert O.level_sizes(1024, 436, 5) == [(1024, 436), (512, 218), (256, 109), (128, 54), (64, 27), (32, 13)]


def test_p15_upsampling_a_constant_field():
    U = torch.stack([torch.full((6, 7), 0.75, dtype=F64), torch.full((6, 7), -2.0, dtype=F64)])
    for s in (1, 2, 3):
        up = O.upsample(U, 7 * 2 ** s + 1, 6 * 2 ** s + 3, s, params())
        assert torch.equal(up[0], torch.full_like(up[0], 0.75 * 2 ** s))
        assert torch.equal(up[1], torch.full_like(up[1], -2.0 * 2 ** s))


# ------------------------------------------------------------------ P16 ------
def test_p16_transposing_the_frames_transposes_the_flow():
    from paper_1603_03590_amd import synth
    pr = synth.smooth_bump_pair(96, 96, 5.0, 16)
    I0 = torch.from_numpy(pr.I0).to(F64)
    I1 = torch.from_numpy(pr.I1).to(F64)
    p = params(refine=False, coarsest_scale=3, finest_scale=0)
    U = O.dis_flow(I0, I1, p)
    Ut = O.dis_flow(I0.T.contiguous(), I1.T.contiguous(), p)
    assert (Ut[0].T - U[1]).abs().max() < 1e-9
    assert (Ut[1].T - U[0]).abs().max() < 1e-9


# ------------------------------------------------------------ gradient -------
def test_oracle_autograd_matches_finite_differences():
    """The oracle's autograd gradient (the reference for the adjoint) agrees
    with central differences of the oracle itself."""
    from paper_1603_03590_amd import synth
    pr = synth.smooth_bump_pair(32, 32, 2.0, 17)
    I0 = torch.from_numpy(pr.I0).to(F64).requires_grad_(True)
    I1 = torch.from_numpy(pr.I1).to(F64).requires_grad_(True)
    gt = torch.from_numpy(pr.flow)
    p = params(coarsest_scale=2, finest_scale=0, gn_iters=6, var_outer=2)

    def loss(a, b):
        return O.endpoint_error(O.dis_flow(a, b, p), gt).mean()

    L = loss(I0, I1)
    g0, g1 = torch.autograd.grad(L, (I0, I1))
    rng = np.random.default_rng(18)
    hstep = 1e-6
    for img, g in ((I0, g0), (I1, g1)):
        for _ in range(6):
            y, x = rng.integers(2, 30, 2)
            e = torch.zeros_like(img)
            e[y, x] = hstep
            with torch.no_grad():
                fd = (loss(I0 + (e if img is I0 else 0), I1 + (e if img is I1 else 0))
                      - loss(I0 - (e if img is I0 else 0), I1 - (e if img is I1 else 0))) / (2 * hstep)
            assert abs(float(fd) - float(g[y, x])) < 1e-6 + 1e-4 * abs(float(fd)), (float(fd), float(g[y, x]))


# ------------------------------------------------------- extra pins ---------
def test_p8_reset_threshold_is_the_patch_size():
    """A patch that ends between theta_ps/2 and theta_ps from its start keeps
    its result; the reset needs more than theta_ps (Sec. 2.2 step 4)."""
    t = (6.0, 1.5)
    J0 = 255 * analytic_texture(64, 64, seed=19, min_period=20.0, n=6)
    J1 = 255 * analytic_texture(64, 64, shift=t, seed=19, min_period=20.0, n=6)
    Gx, Gy = O.sobel8(J0)
    x0, y0 = torch.tensor([28]), torch.tensor([28])
    res = O.inverse_search(J0, Gx, Gy, J1, x0, y0, torch.zeros(1, 2, dtype=F64), params(gn_iters=100))
    moved = float(res.u_search[0].norm())
    assert 4.0 < moved < 8.0
    assert not res.reset.any()
    assert (res.u[0] - torch.tensor(t, dtype=F64)).norm() < 0.05


def test_p15_refinement_derivatives_exact_on_quadratics():
    """Central differences are exact for quadratics, so on I0 = q0(x, y),
    I1 = q1(x, y) with U = 0 every linearisation term of Sec. 2.3 equals the
    analytic derivative away from the border."""
    h, w = 20, 24
    yy, xx = torch.meshgrid(torch.arange(h, dtype=F64), torch.arange(w, dtype=F64), indexing="ij")
    q0 = 0.3 * xx * xx - 0.2 * xx * yy + 0.1 * yy * yy + 2 * xx - yy + 50
    q1 = 0.25 * xx * xx + 0.15 * xx * yy - 0.12 * yy * yy - xx + 3 * yy + 40
    t = O.refine_linearise(q0, q1, torch.zeros(2, h, w, dtype=F64))
    ib = lambda f: f[2:-2, 2:-2]
    # mean image (q0+q1)/2 = 0.275 x^2 - 0.025 xy - 0.01 y^2 + 0.5 x + y + 45
    assert torch.allclose(ib(t.Ix), ib(0.55 * xx - 0.025 * yy + 0.5), atol=1e-10)
    assert torch.allclose(ib(t.Iy), ib(-0.025 * xx - 0.02 * yy + 1.0), atol=1e-10)
    assert torch.allclose(ib(t.Iz), ib(q1 - q0), atol=1e-10)
    assert torch.allclose(ib(t.Ixx), torch.full_like(ib(xx), 0.55), atol=1e-10)
    assert torch.allclose(ib(t.Ixy), torch.full_like(ib(xx), -0.025), atol=1e-10)
    assert torch.allclose(ib(t.Iyy), torch.full_like(ib(xx), -0.02), atol=1e-10)
    # d/dx (q1 - q0) and d/dy (q1 - q0)
    assert torch.allclose(ib(t.Ixz), ib(-0.1 * xx + 0.35 * yy - 3.0), atol=1e-10)
    assert torch.allclose(ib(t.Iyz), ib(0.35 * xx - 0.44 * yy + 4.0), atol=1e-10)


def test_p16_red_pixels_relax_first():
    """R16: the first half sweep moves only pixels with x + y even."""
    J0, J1, U = _level_problem(seed=20, h=9, w=11)
    p = params()
    t = O.refine_linearise(J0, J1, U)
    zero = torch.zeros_like(U[0])
    sys = O.sor_system(t, U, zero, zero, p)
    seen = []
    O.sor_sweeps(sys, U, zero, zero, 1, p.sor_omega, lambda a, b: seen.append((a.clone(), b.clone())))
    yy, xx = torch.meshgrid(torch.arange(9), torch.arange(11), indexing="ij")
    black = (xx + yy) % 2 == 1
    du1, dv1 = seen[0]
    assert torch.count_nonzero(du1[black]) == 0 and torch.count_nonzero(dv1[black]) == 0
    assert torch.count_nonzero(du1[~black]) > 0
    du2, _ = seen[1]
    assert torch.equal(du2[~black], du1[~black])


def test_refinement_pulls_a_perturbed_flow_towards_the_truth():
    """On a globally translated pair, refining U = t + e reduces the error
    (checks the sign of the temporal derivatives)."""
    t = (2.25, -1.5)
    J0 = 255 * analytic_texture(48, 56, seed=21, min_period=12.0, n=16)
    J1 = 255 * analytic_texture(48, 56, shift=t, seed=21, min_period=12.0, n=16)
    U = torch.stack([torch.full((48, 56), t[0] + 0.3, dtype=F64), torch.full((48, 56), t[1] - 0.2, dtype=F64)])
    e0 = math.hypot(0.3, 0.2)
    errs = []
    for n_outer in (1, 3, 6):
        R = O.refine(J0, J1, U, n_outer, params())
        errs.append(float(torch.sqrt((R[0] - t[0]) ** 2 + (R[1] - t[1]) ** 2)[6:-6, 6:-6].mean()))
    assert errs[0] < e0 and errs[1] < errs[0] and errs[2] < 0.6 * e0, errs


# --------------------------------------------- robust norms (App. B iii) ----
def test_r17_squared_transform_is_the_l1_and_huber_penalty():
    """App. B iii: after squaring, the transformed residual is the L1 norm
    |e|, or the Huber penalty (quadratic inside b, linear outside, C1 at b;
    here twice the textbook Huber function b |e| - b^2/2 beyond b)."""
    pos = torch.linspace(0.0, 30.0, 3001, dtype=F64)
    e = torch.cat([-pos.flip(0), pos[1:]])           # exactly symmetric grid
    l1 = O.robust_residual(e, params(norm="l1"))
    assert torch.allclose(l1 ** 2, e.abs(), rtol=0, atol=1e-12)
    b = 2.5
    hub = O.robust_residual(e, params(norm="huber", huber_b=b))
    textbook = torch.where(e.abs() <= b, 0.5 * e * e, b * (e.abs() - 0.5 * b))
    assert torch.allclose(hub ** 2, 2.0 * textbook, rtol=0, atol=1e-10)
    # odd, sign-preserving, continuous at the threshold; L2 untouched
    for r in (l1, hub):
        assert torch.allclose(r, -torch.flip(r, [0]), atol=1e-12)
        assert bool(((r >= 0) == (e >= 0)).all())
    near = torch.tensor([b - 1e-9, b + 1e-9], dtype=F64)
    h = O.robust_residual(near, params(norm="huber", huber_b=b))
    assert abs(float(h[1] - h[0])) < 1e-6
    assert torch.equal(O.robust_residual(e, params()), e)


def test_r17_zero_residual_is_a_fixed_point_and_wide_huber_is_l2():
    """A zero residual is a fixed point of every transform (an integer shift
    makes the bilinear warp exact), and a Huber threshold above every
    residual leaves the search exactly the L2 one of Sec. 2.1.  (Whether the
    transformed iteration is more robust to outliers depends on the case --
    the mean normalisation spreads an outlier's offset over the patch; the
    paper found the gain not worth the slower convergence.)"""
    t = (2.0, -1.0)
    J0 = 255 * analytic_texture(64, 64, seed=21, min_period=14.0, n=8)
    J1 = 255 * analytic_texture(64, 64, shift=t, seed=21, min_period=14.0, n=8)
    Gx, Gy = O.sobel8(J0)
    x0, y0 = torch.tensor([24, 8]), torch.tensor([24, 30])
    exact = torch.tensor([[t[0], t[1]], [t[0], t[1]]], dtype=F64)
    for norm in ("l2", "l1", "huber"):
        res = O.inverse_search(J0, Gx, Gy, J1, x0, y0, exact.clone(), params(norm=norm, huber_b=1.0, gn_iters=3))
        assert float((res.u - exact).norm()) < 1e-12, norm
    init = torch.zeros(2, 2, dtype=F64)
    l2 = O.inverse_search(J0, Gx, Gy, J1, x0, y0, init, params(gn_iters=10))
    wide = O.inverse_search(J0, Gx, Gy, J1, x0, y0, init, params(norm="huber", huber_b=1e9, gn_iters=10))
    assert torch.equal(l2.u_search, wide.u_search)
    # the L1 search closes most of a one-pixel start error, then hovers
    # around the shift: sqrt|e| has an unbounded slope at zero, so the
    # least-squares step overshoots small residuals
    l1 = O.inverse_search(J0, Gx, Gy, J1, x0, y0, exact + 1.0, params(norm="l1", gn_iters=60))
    assert float((l1.u_search - exact).abs().max()) < 0.25


# ------------------------------------------------------ stereo (App. I) -----
def test_r18_stereo_recovers_horizontal_shifts_with_a_zero_vertical_plane():
    """With the vertical degree of freedom removed, an integer horizontal
    shift is a fixed point of the search, the 1-D step from a nearby start
    closes the gap like the 2-D one on the same pair, and the whole pipeline
    returns a flow whose vertical plane is exactly zero."""
    t = (3.0, 0.0)
    J0 = 255 * analytic_texture(64, 64, seed=31, min_period=14.0, n=8)
    J1 = 255 * analytic_texture(64, 64, shift=t, seed=31, min_period=14.0, n=8)
    Gx, Gy = O.sobel8(J0)
    x0, y0 = torch.tensor([24, 8, 40]), torch.tensor([24, 30, 12])
    exact = torch.tensor([[3.0, 0.0]] * 3, dtype=F64)
    res = O.inverse_search(J0, Gx, Gy, J1, x0, y0, exact.clone(), params(stereo=True, gn_iters=3))
    assert float((res.u - exact).norm()) < 1e-12
    start = exact + torch.tensor([[0.6, 0.0]] * 3, dtype=F64)
    r1 = O.inverse_search(J0, Gx, Gy, J1, x0, y0, start, params(stereo=True, gn_iters=30))
    assert float((r1.u_search - exact).abs().max()) < 1e-6
    assert bool((r1.u_search[:, 1] == 0).all())
    from paper_1603_03590_amd import synth
    pr = synth.smooth_bump_pair(96, 80, 4.0, 32, horizontal=True)
    assert np.abs(pr.flow[1]).max() == 0.0
    U = O.dis_flow(torch.from_numpy(pr.I0), torch.from_numpy(pr.I1),
                   params(stereo=True, coarsest_scale=2, finest_scale=0, gn_iters=8, var_outer=2))
    assert bool((U[1] == 0).all())
    assert float(O.endpoint_error(U, torch.from_numpy(pr.flow)).mean()) < 0.5


# ------------------------ forward-backward consistency (App. B ii, R19) ----
def test_r19_swap_symmetry_and_reduction_to_the_plain_method():
    """Swapping the frames swaps the two flows bit for bit, and without the
    other direction's votes the forward flow is the plain method's."""
    from paper_1603_03590_amd import synth
    pr = synth.smooth_bump_pair(96, 80, 4.0, 40)
    a, b = torch.from_numpy(pr.I0), torch.from_numpy(pr.I1)
    p = params(coarsest_scale=2, finest_scale=0, gn_iters=8, var_outer=2)
    Uf, Ub = O.dis_flow_fb(a, b, p)
    Ub2, Uf2 = O.dis_flow_fb(b, a, p)
    assert torch.equal(Uf, Uf2) and torch.equal(Ub, Ub2)
    Un, _ = O.dis_flow_fb(a, b, p, merge=False)
    assert torch.equal(Un, O.dis_flow(a, b, p))
    # consistent votes help a little on this pair (the paper's extension)
    gt = torch.from_numpy(pr.flow)
    assert float(O.endpoint_error(Uf, gt).mean()) < float(O.endpoint_error(Un, gt).mean())


def test_r19_merged_votes_of_a_consistent_translation():
    """Own patches at u = t and the other direction's patches at -t (zero
    residuals) densify to exactly t wherever they vote."""
    J = 255 * analytic_texture(40, 48, seed=41, min_period=10.0, n=6)
    p = params(patch_size=8, overlap=0.5)
    x0, y0, nx, ny = O.patch_grid(48, 40, p)
    N = x0.numel()
    t = torch.tensor([2.0, -1.0], dtype=F64)
    u_own = t.expand(N, 2).clone()
    u_oth = (-t).expand(N, 2).clone()
    d_own = torch.zeros(N, 64, dtype=F64)
    md = torch.zeros(N, dtype=F64)
    U = O.merged_densify(J, J, x0, y0, u_own, d_own, u_oth, md, p)
    assert torch.equal(U[0], torch.full_like(U[0], 2.0)) and torch.equal(U[1], torch.full_like(U[1], -1.0))


def test_r19_displaced_patch_coverage_and_residual_by_hand():
    """One other-direction patch at corner (8, 8) displaced by (0.5, 0): it
    votes on the pixels x with x - 0.5 in [8, 15] (columns 9..15, rows 8..15)
    with the residual Jref(x) - T(x - 0.5) - md; on a linear ramp both frames
    equal, T(x - 0.5) is the ramp half a pixel back."""
    H, Wd = 32, 32
    ramp = torch.arange(Wd, dtype=F64).expand(H, Wd).clone() * 3.0    # Jother(x, y) = 3x
    Jref = ramp.clone()
    p = params(patch_size=8, overlap=0.5)
    x0 = torch.tensor([0]); y0 = torch.tensor([0])              # one own patch far away
    u_own = torch.zeros(1, 2, dtype=F64); d_own = torch.zeros(1, 64, dtype=F64)
    xo, yo = torch.tensor([8]), torch.tensor([8])
    u_oth = torch.tensor([[0.5, 0.0]], dtype=F64)
    md = torch.tensor([0.25], dtype=F64)
    # own patch covers rows/cols 0..7 only: elsewhere only the other patch votes
    U = O.merged_densify_pairs(Jref, ramp, x0, y0, u_own, d_own, xo, yo, u_oth, md, p)
    covered = torch.zeros(H, Wd, dtype=torch.bool)
    covered[8:16, 9:16] = True
    assert torch.equal(U[0][covered], torch.full((int(covered.sum()),), -0.5, dtype=F64))
    assert bool(torch.isnan(U[0][~covered & (torch.arange(H)[:, None] > 7)]).all())
    # the weight of a covered pixel: d = 3x - 3(x - 0.5) - 0.25 = 1.25 -> 1/1.25
    Z = O.merged_densify_pairs(Jref, ramp, x0, y0, u_own, d_own, xo, yo, u_oth, md, p, want_z=True)
    assert torch.allclose(Z[covered], torch.full((int(covered.sum()),), 1 / 1.25, dtype=F64), rtol=0, atol=1e-15)


def test_r19_patches_displaced_off_the_level_vote_nowhere():
    """Other-direction patches whose displaced squares lie wholly outside the
    level (right, below, left, above) leave Eq. (3) over the own patches
    unchanged, bit for bit; one that overlaps the border by a column votes on
    that column only."""
    H, Wd = 24, 24
    J = 255 * analytic_texture(H, Wd, seed=42, min_period=8.0, n=5)
    p = params(patch_size=8, overlap=0.5)
    x0, y0, _, _ = O.patch_grid(Wd, H, p)
    N = x0.numel()
    g = torch.Generator().manual_seed(5)
    u_own = torch.rand(N, 2, generator=g, dtype=F64)
    d_own = torch.rand(N, 64, generator=g, dtype=F64) * 4 - 2
    xo = torch.tensor([0, 0, 16, 16]); yo = torch.tensor([0, 16, 0, 16])
    u_oth = torch.tensor([[30.0, 0.0], [0.0, 9.5], [-24.2, 0.0], [0.0, -23.01]], dtype=F64)
    md = torch.zeros(4, dtype=F64)
    ref = O.merged_densify_pairs(J, J, x0, y0, u_own, d_own, xo[:0], yo[:0], u_oth[:0], md[:0], p)
    U = O.merged_densify_pairs(J, J, x0, y0, u_own, d_own, xo, yo, u_oth, md, p)
    assert torch.equal(U, ref)
    # corner (16, 0) displaced by (-23, 0): x - (-23) in [16, 23] -> column 0 only
    U1 = O.merged_densify_pairs(J, J, x0, y0, u_own, d_own, xo[2:3], yo[2:3],
                                torch.tensor([[-23.0, 0.0]], dtype=F64), md[:1], p)
    changed = (U1 != ref).any(0)
    assert bool(changed[:8, 0].all()) and not bool(changed[:, 1:].any()) and not bool(changed[8:, :].any())


# ------------------------------------------------------------------ R20 ------
def _colour_pair(w, h, seed, disp=4.0):
    from paper_1603_03590_amd import synth
    pr = synth.smooth_bump_pair(w, h, disp, seed, channels=3)
    return torch.from_numpy(pr.I0).double(), torch.from_numpy(pr.I1).double(), pr


def test_r20_zero_channels_reduce_to_the_grey_method():
    """Two all-zero channels add exact zeros to H', to the right-hand side
    and to both data terms of the refinement, and the channel norm of Eq. (3)
    is then sqrt(d^2) = |d| (torch's vectorised CPU sqrt is not always
    correctly rounded, so the norm may differ from |d| in the last bit): the
    colour method is the grey one to rounding."""
    a, b, _ = _colour_pair(96, 80, 50)
    z = torch.zeros_like(a[0])
    for kw in (dict(), dict(norm="l1"), dict(refine=False, residual="raw")):
        p = params(coarsest_scale=2, gn_iters=8, var_outer=2, **kw)
        Uc = O.dis_flow_colour(torch.stack([a[0], z, z]), torch.stack([b[0], z, z]), p)
        assert torch.allclose(Uc, O.dis_flow(a[0], b[0], p), rtol=0, atol=1e-12), kw
    # the search alone involves no square root: bit for bit
    p = params(gn_iters=8, norm="l1")
    x0, y0, _, _ = O.patch_grid(96, 80, p)
    ui = torch.full((x0.numel(), 2), 0.3, dtype=F64)
    J0, J1 = 255 * a[0], 255 * b[0]
    rc = O.colour_search(torch.stack([J0, z, z]), torch.stack([J1, z, z]), x0, y0, ui, p)
    Gx, Gy = O.sobel8(J0)
    rg = O.inverse_search(J0, Gx, Gy, J1, x0, y0, ui, p)
    assert torch.equal(rc.u, rg.u) and torch.equal(rc.d[0], rg.d) and not bool(rc.d[1:].any())


def test_r20_three_equal_channels_triple_the_normal_equations():
    """Channels (J, J, J): H' and the right-hand side are three times the
    grey ones, so the step solves (3H + lambda I) du = 3b, the grey step with
    lambda / 3.  A search that dropped or doubled a channel fails this."""
    a, b, _ = _colour_pair(64, 64, 51)
    J0, J1 = 255 * a[0], 255 * b[0]
    p = params(gn_iters=6)
    x0, y0, _, _ = O.patch_grid(64, 64, p)
    g = torch.Generator().manual_seed(3)
    ui = torch.rand(x0.numel(), 2, generator=g, dtype=F64) * 2 - 1
    rc = O.colour_search(torch.stack([J0, J0, J0]), torch.stack([J1, J1, J1]), x0, y0, ui, p)
    Gx, Gy = O.sobel8(J0)
    rg = O.inverse_search(J0, Gx, Gy, J1, x0, y0, ui, O.with_params(p, hessian_lambda=p.hessian_lambda / 3))
    assert torch.allclose(rc.u, rg.u, rtol=0, atol=1e-9)
    assert torch.allclose(rc.hessian, 3 * rg.hessian, rtol=1e-15, atol=0)
    for c in range(3):
        assert torch.allclose(rc.d[c], rg.d, rtol=0, atol=1e-9)


def test_r20_channel_norm_of_the_densification_weight_by_hand():
    """Two patches on the same square; per-channel residuals (3, 4, 0) and
    (0.5, 0, 0): weights 1/5 and 1, so U = (u1/5 + u2) / (1/5 + 1)."""
    p = params(patch_size=4)
    x0 = torch.tensor([0, 0]); y0 = torch.tensor([0, 0])
    u = torch.tensor([[2.0, -1.0], [0.5, 0.25]], dtype=F64)
    d = torch.zeros(3, 2, 16, dtype=F64)
    d[0, 0], d[1, 0] = 3.0, 4.0
    d[0, 1] = 0.5
    U, Z = O.colour_densify(4, 4, x0, y0, u, d, p)
    assert torch.allclose(Z, torch.full((4, 4), 1.2, dtype=F64), rtol=0, atol=1e-15)
    assert torch.allclose(U[0], torch.full((4, 4), (2.0 / 5 + 0.5) / 1.2, dtype=F64), rtol=0, atol=1e-15)
    assert torch.allclose(U[1], torch.full((4, 4), (-1.0 / 5 + 0.25) / 1.2, dtype=F64), rtol=0, atol=1e-15)


def test_r20_one_robust_function_over_the_channel_sum():
    """Channels (J, J, J) in the refinement: each data energy triples inside
    one robust function, so the frozen system is the grey one with delta and
    gamma times sqrt(3) and eps / sqrt(3) (the data part; the smoothness
    weight keeps eps).  A robust function per channel would give 3 delta and
    eps instead."""
    a, b, _ = _colour_pair(48, 40, 52)
    J0, J1 = 255 * a[0], 255 * b[0]
    g = torch.Generator().manual_seed(4)
    U = torch.rand(2, 40, 48, generator=g, dtype=F64) * 2 - 1
    du = torch.rand(40, 48, generator=g, dtype=F64) * 0.2
    dv = torch.rand(40, 48, generator=g, dtype=F64) * 0.2
    p = params()
    t = O.refine_linearise(J0, J1, U)
    ts = O.colour_linearise(torch.stack([J0, J0, J0]), torch.stack([J1, J1, J1]), U)
    sc = O.colour_sor_system(ts, U, du, dv, p)
    r3 = math.sqrt(3.0)
    sg = O.sor_system(t, U, du, dv, O.with_params(p, delta=r3 * p.delta, gamma=r3 * p.gamma, eps=p.eps / r3))
    for name in ("A11", "A12", "A22", "b1", "b2"):
        x, y = getattr(sc, name), getattr(sg, name)
        assert torch.allclose(x, y, rtol=1e-12, atol=1e-12 * float(y.abs().max())), name


def test_r20_channel_order_does_not_matter_and_integer_shift_is_fixed():
    """Permuting the channels permutes only the order of the channel sums;
    an integer shift of all channels is a fixed point of the colour search."""
    a, b, pr = _colour_pair(96, 80, 53)
    p = params(coarsest_scale=2, gn_iters=8, var_outer=2)
    U = O.dis_flow_colour(a, b, p)
    Up = O.dis_flow_colour(a[[2, 0, 1]], b[[2, 0, 1]], p)
    assert torch.allclose(U, Up, rtol=0, atol=1e-6)
    # using one channel only (or the grey frame) is a different method
    assert float((U - O.dis_flow(a[0], b[0], p)).abs().max()) > 1e-3
    J0 = 255 * a
    J1 = torch.roll(J0, shifts=(1, 2), dims=(1, 2))        # J1(x + (2, 1)) = J0(x) away from the wrap
    p8 = params(patch_size=8, overlap=0.5)
    x0, y0, _, _ = O.patch_grid(96, 80, p8)
    keep = (x0 >= 2) & (x0 + 8 + 2 <= 96) & (y0 >= 1) & (y0 + 8 + 1 <= 80)
    ui = torch.tensor([[2.0, 1.0]], dtype=F64).expand(int(keep.sum()), 2).clone()
    r = O.colour_search(J0, J1, x0[keep], y0[keep], ui, p8)
    assert torch.equal(r.u, ui)


# ----------------------------------------- sample positions and borders -----
def _affine_field(h, w, a, b):
    """u(x, y) = a0 x + a1 y + a2, v(x, y) = b0 x + b1 y + b2 on the integer
    grid of an h x w level (bilinear interpolation reproduces it exactly
    between the samples)."""
    yy, xx = torch.meshgrid(torch.arange(h, dtype=F64), torch.arange(w, dtype=F64), indexing="ij")
    return torch.stack([a[0] * xx + a[1] * yy + a[2], b[0] * xx + b[1] * yy + b[2]])


def test_r7_initialisation_samples_the_coarser_flow_at_half_the_patch_centre():
    """Sec. 2.2 step 2: a patch starts from twice the coarser flow at its
    centre mapped to the coarser scale.  On an affine coarse field the value
    is known by hand for every patch whose sample point is inside the field;
    a corner instead of the centre, a missing factor 2 or a wrong mapping
    each move it."""
    a, b = (0.5, 0.25, 1.0), (-0.125, 0.75, -2.0)
    Un = _affine_field(20, 24, a, b)
    p = params(patch_size=8)
    # corner (10, 6): centre (13.5, 9.5); literal mapping samples (6.75, 4.75)
    x0, y0 = torch.tensor([10, 0, 30]), torch.tensor([6, 4, 22])
    u = O.init_displacements(Un, x0, y0, p)
    assert u[0, 0].item() == 2.0 * (0.5 * 6.75 + 0.25 * 4.75 + 1.0) == 11.125
    assert u[0, 1].item() == 2.0 * (-0.125 * 6.75 + 0.75 * 4.75 - 2.0) == 1.4375
    # pixel-centre mapping samples ((13.5 + 0.5) / 2 - 0.5, (9.5 + 0.5) / 2 - 0.5) = (6.5, 4.5)
    uc = O.init_displacements(Un, x0, y0, O.with_params(p, init_map="pixel_centre"))
    assert uc[0, 0].item() == 2.0 * (0.5 * 6.5 + 0.25 * 4.5 + 1.0) == 10.75
    assert uc[0, 1].item() == 2.0 * (-0.125 * 6.5 + 0.75 * 4.5 - 2.0) == 1.125
    # every interior patch of a grid: twice the affine field at the sample point
    x0g, y0g, _, _ = O.patch_grid(40, 36, p)
    for mode, m in (("literal", lambda c: c / 2.0), ("pixel_centre", lambda c: (c + 0.5) / 2.0 - 0.5)):
        ug = O.init_displacements(Un, x0g, y0g, O.with_params(p, init_map=mode))
        qx, qy = m(x0g.double() + 3.5), m(y0g.double() + 3.5)
        assert float(qx.max()) <= 23 and float(qy.max()) <= 19
        assert torch.allclose(ug[:, 0], 2.0 * (a[0] * qx + a[1] * qy + a[2]), atol=1e-12, rtol=0)
        assert torch.allclose(ug[:, 1], 2.0 * (b[0] * qx + b[1] * qy + b[2]), atol=1e-12, rtol=0)
    # a 12x12 patch at corner (0, 4): centre (5.5, 9.5), sample (2.75, 4.75)
    u12 = O.init_displacements(Un, torch.tensor([0]), torch.tensor([4]), params(patch_size=12))
    assert u12[0, 0].item() == 2.0 * (0.5 * 2.75 + 0.25 * 4.75 + 1.0) == 7.125
    # a sample point past the coarser field's last column (centre 47.5 ->
    # 23.75 on a 24-wide field) takes the border column's value (R8)
    ub = O.init_displacements(Un, torch.tensor([44]), torch.tensor([6]), p)
    assert ub[0, 0].item() == 2.0 * (0.5 * 23 + 0.25 * 4.75 + 1.0)


def test_sec31_upscaling_of_an_affine_field():
    """End of Sec. 3.1: the finest computed flow is interpolated bilinearly to
    the full resolution and its vectors scaled by 2^s.  An affine level field
    A x + t becomes A x + 2^s t at every output pixel whose sample point lies
    inside the level (literal mapping x / 2^s), and A (x + 1/2 - 2^s / 2) + 2^s t
    under the pixel-centre mapping; a wrong sample point or scale fails."""
    a, b = (0.5, -0.25, 1.5), (0.125, 0.375, -0.75)
    hs, ws = 7, 9
    U = _affine_field(hs, ws, a, b)
    for s in (1, 2, 3):
        f = 2 ** s
        w, h = ws * f, hs * f
        yy, xx = torch.meshgrid(torch.arange(h, dtype=F64), torch.arange(w, dtype=F64), indexing="ij")
        up = O.upsample(U, w, h, s, params())
        inside = (xx <= (ws - 1) * f) & (yy <= (hs - 1) * f)
        ex_u = a[0] * xx + a[1] * yy + f * a[2]
        ex_v = b[0] * xx + b[1] * yy + f * b[2]
        assert torch.allclose(up[0][inside], ex_u[inside], atol=1e-12, rtol=0)
        assert torch.allclose(up[1][inside], ex_v[inside], atol=1e-12, rtol=0)
        # one pixel by hand: s = 1, pixel (x=3, y=5) samples (1.5, 2.5):
        if s == 1:
            assert up[0][5, 3].item() == 2.0 * (0.5 * 1.5 - 0.25 * 2.5 + 1.5)
        upc = O.upsample(U, w, h, s, O.with_params(params(), init_map="pixel_centre"))
        qx, qy = (xx + 0.5) / f - 0.5, (yy + 0.5) / f - 0.5
        inside_c = (qx >= 0) & (qy >= 0) & (qx <= ws - 1) & (qy <= hs - 1)
        ex_uc = a[0] * (xx + 0.5 - f / 2) + a[1] * (yy + 0.5 - f / 2) + f * a[2]
        ex_vc = b[0] * (xx + 0.5 - f / 2) + b[1] * (yy + 0.5 - f / 2) + f * b[2]
        assert torch.allclose(upc[0][inside_c], ex_uc[inside_c], atol=1e-12, rtol=0)
        assert torch.allclose(upc[1][inside_c], ex_vc[inside_c], atol=1e-12, rtol=0)


def test_sec23_data_term_normalisers_by_hand():
    """Sec. 2.3: beta_0 = 1 / (|grad_2 I|^2 + 0.01) from the first spatial
    derivatives, beta_x = 1 / (I_xx^2 + I_xy^2 + 0.01) from the gradient of
    I_x and beta_y = 1 / (I_xy^2 + I_yy^2 + 0.01) from the gradient of I_y.
    On quadratic frames (central differences exact) the second derivatives of
    the mean image are the constants 0.55, -0.025 and -0.02, so the values are
    fixed by hand; swapping I_xy and I_yy, or I_xx and I_yy, changes them."""
    h, w = 20, 24
    yy, xx = torch.meshgrid(torch.arange(h, dtype=F64), torch.arange(w, dtype=F64), indexing="ij")
    q0 = 0.3 * xx * xx - 0.2 * xx * yy + 0.1 * yy * yy + 2 * xx - yy + 50
    q1 = 0.25 * xx * xx + 0.15 * xx * yy - 0.12 * yy * yy - xx + 3 * yy + 40
    t = O.refine_linearise(q0, q1, torch.zeros(2, h, w, dtype=F64))
    ib = lambda f: f[2:-2, 2:-2]
    bx = 1.0 / (0.3025 + 0.000625 + 0.01)        # 0.55^2 + 0.025^2 + 0.01
    by = 1.0 / (0.000625 + 0.0004 + 0.01)        # 0.025^2 + 0.02^2 + 0.01
    assert torch.allclose(ib(t.bx), torch.full_like(ib(xx), bx), rtol=1e-12, atol=0)
    assert torch.allclose(ib(t.by), torch.full_like(ib(xx), by), rtol=1e-12, atol=0)
    # pixel (x=10, y=8): I_x = 0.55*10 - 0.025*8 + 0.5 = 5.8, I_y = -0.25 - 0.16 + 1 = 0.59
    assert abs(t.b0[8, 10].item() - 1.0 / (5.8 ** 2 + 0.59 ** 2 + 0.01)) < 1e-15
    assert abs(t.b0[8, 10].item() - 1.0 / 33.9981) < 1e-15
    # the values a plausible slip would give are different
    assert abs(bx - 1.0 / (0.3025 + 0.0004 + 0.01)) > 1e-3 and abs(by - 1.0 / (0.000625 + 0.3025 + 0.01)) > 1


def test_r8_bilinear_clamps_at_the_frame_border_by_hand():
    """R8: pixel values sit at integer coordinates and every tap index is
    clamped into the image.  Values by hand on a 3 x 4 image."""
    img = torch.tensor([[1., 2., 4., 8.],
                        [16., 32., 64., 128.],
                        [3., 5., 7., 11.]], dtype=F64)
    pts = [
        # (x, y) -> value
        ((-0.5, 1.0), 16.0),                     # left of the frame: column 0
        ((-3.25, 0.5), 0.5 * 1.0 + 0.5 * 16.0),  # far left, between rows 0 and 1
        ((3.25, 1.0), 128.0),                    # right of the last column
        ((5.0, 2.0), 11.0),                      # right, bottom row
        ((1.5, -2.7), 0.5 * (2.0 + 4.0)),        # above the frame: row 0
        ((2.0, 2.5), 7.0),                       # below the last row
        ((-1.0, -1.0), 1.0), ((-7.5, 9.0), 3.0), ((4.5, -0.5), 8.0), ((3.0, 2.0), 11.0),   # corners
        ((2.5, 1.75), 0.25 * 0.5 * (64.0 + 128.0) + 0.75 * 0.5 * (7.0 + 11.0)),   # interior
        ((0.25, 0.5), 0.5 * (0.75 * 1.0 + 0.25 * 2.0) + 0.5 * (0.75 * 16.0 + 0.25 * 32.0)),
    ]
    x = torch.tensor([p[0][0] for p in pts], dtype=F64)
    y = torch.tensor([p[0][1] for p in pts], dtype=F64)
    got = O.bilinear(img, x, y)
    for k, (_, v) in enumerate(pts):
        assert got[k].item() == v, (pts[k], got[k].item())
