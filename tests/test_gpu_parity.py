"""GPU path against the FP64 oracle, through the C ABI (ctypes binding).

Every GPU test prints its case before it touches the device.
"""
import sys

import numpy as np
import pytest
import torch

from dis_cases import PARITY_EPE_REL, PARITY_FRAC, oracle_flow, oracle_params, pair, parity
from paper_1603_03590_amd import DIS, DisError, params, _lib

pytestmark = pytest.mark.gpu

N_TILES = 13   # refinement tile ids the library knows


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_flow(I0, I1, p, max_wh=None, keep=False):
    h, w = I0.shape[-2:]
    mw, mh = max_wh or (w, h)
    d = DIS(p, mw, mh)
    dt = d.dtype
    t0 = torch.from_numpy(I0).to(dt).cuda()
    t1 = torch.from_numpy(I1).to(dt).cuda()
    out = d.flow(t0, t1)
    torch.cuda.synchronize()
    U = out.cpu().numpy().astype(np.float64)
    if keep:
        return U, d
    d.close()
    return U


CASES = [
    # name, generator (kind, w, h, max displacement, seed), preset, overrides
    ("c1_bump_256x192", ("bump", 256, 192, 8.0, 1), 101, {}),
    ("c2a_layered_1024x436", ("layered", 1024, 436, 100.0, 2), 102, {}),
    ("c2b_layered_1024x436", ("layered", 1024, 436, 100.0, 2), 103, {}),
    ("c5_bump_512x256", ("bump", 512, 256, 16.0, 2000), 105, {}),
    ("ragged_203x149_norefine", ("layered", 203, 149, 20.0, 7), 103,
     dict(coarsest_scale=3, finest_scale=0, refine=0)),
    ("ragged_203x149_sf1", ("layered", 203, 149, 20.0, 8), 103, dict(coarsest_scale=3, finest_scale=1)),
    ("c3_small_320x240", ("layered", 320, 240, 60.0, 9), 104, dict(coarsest_scale=3, gn_iters=64, var_outer=2)),
    ("op1_norefine_640x480", ("layered", 640, 480, 40.0, 10), 1, {}),
    ("pixel_centre_raw_300x200", ("bump", 300, 200, 10.0, 11), 105, dict(flags=0x4 | 0x8)),
    ("io_f64_256x192", ("bump", 256, 192, 8.0, 12), 101, dict(flags=0x10)),
    ("ps12_ov05_288x216", ("bump", 288, 216, 10.0, 13), 105, dict(patch_size=12, overlap=0.5, var_inner=7)),
    ("ps6_ov0_auto_320x96", ("layered", 320, 96, 12.0, 14), 103,
     dict(patch_size=6, overlap=0.0, coarsest_scale=-1, finest_scale=0)),
    ("op3_1024x436", ("layered", 1024, 436, 100.0, 15), 3, dict(gn_iters=16)),
    # rectified stereo, horizontal displacement only (App. I; theta_it halved)
    ("stereo_hbump_256x192", ("hbump", 256, 192, 8.0, 17), 101, dict(flags=0x20, gn_iters=4)),
    ("stereo_hbump_640x480_op2", ("hbump", 640, 480, 20.0, 18), 2, dict(flags=0x20, gn_iters=6)),
    # robust error norms of the search (App. B iii)
    ("l1_bump_256x192", ("bump", 256, 192, 8.0, 1), 101, dict(norm=1)),
    ("huber_layered_512x256", ("layered", 512, 256, 40.0, 16), 103, dict(norm=2, huber_b=1.0,
                                                                         coarsest_scale=4, finest_scale=1)),
    # colour frames (App. B i)
    ("colour_bump_256x192", ("cbump", 256, 192, 8.0, 31), 101, dict(flags=0x80)),
    ("colour_bump_512x256_c5", ("cbump", 512, 256, 16.0, 32), 105, dict(flags=0x80)),
    ("colour_ps12_raw_norefine_300x200", ("cbump", 300, 200, 10.0, 33), 105,
     dict(flags=0x80 | 0x8, patch_size=12, refine=0, finest_scale=0, coarsest_scale=3)),
    ("colour_ps4_l1_inner7_203x149", ("cbump", 203, 149, 6.0, 34), 103,
     dict(flags=0x80, patch_size=4, norm=1, var_inner=7, coarsest_scale=3, finest_scale=0)),
    ("colour_stereo_256x192", ("chbump", 256, 192, 8.0, 35), 101, dict(flags=0x80 | 0x20, gn_iters=4)),
    # degenerate sizes: a coarsest level of exactly one patch, a frame of
    # exactly one patch, and a frame one patch high with a ragged width
    ("tiny_16x16_one_patch_coarsest", ("bump", 16, 16, 2.0, 41), 105, dict(coarsest_scale=1, finest_scale=0)),
    ("tiny_8x8_single_patch", ("bump", 8, 8, 2.0, 41), 105, dict(coarsest_scale=0, finest_scale=0)),
    ("tiny_19x11", ("bump", 19, 11, 2.0, 41), 105, dict(coarsest_scale=0, finest_scale=0)),
]


@pytest.mark.parametrize("name,gen,preset,over", CASES, ids=[c[0] for c in CASES])
def test_end_to_end_parity(name, gen, preset, over):
    say(f"[parity] case {name}")
    pr = pair(*gen)
    p = params(preset, **over)
    U_ref, _ = oracle_flow(name, pr.I0, pr.I1, oracle_params(p))
    U = gpu_flow(pr.I0, pr.I1, p)
    frac, erel, dmax = parity(U, U_ref, pr.flow)
    say(f"[parity] {name}: within 1e-2 px {frac:.6f}, mean EPE rel diff {erel:.2e}, max diff {dmax:.2e}")
    if int(p.flags) & 0x20:
        assert np.all(U[1] == 0.0)
    assert frac >= PARITY_FRAC
    assert erel <= PARITY_EPE_REL


def test_level_intermediates_match_oracle():
    """Every level's pyramid image (bitwise), patch initialisation, patch
    displacement, densified and refined flow against the oracle's records."""
    say("[levels] case c1_bump_256x192")
    pr = pair("bump", 256, 192, 8.0, 1)
    p = params(101)
    _, recs = oracle_flow("c1_levels", pr.I0, pr.I1, oracle_params(p), records=True)
    U, d = gpu_flow(pr.I0, pr.I1, p, keep=True)
    try:
        from oracle import dis_oracle as O
        J0 = O.build_pyramid(255.0 * torch.from_numpy(pr.I0).double(), 2)
        for r in recs:
            s = r.s
            g = d.debug_level(s, _lib.DIS_DBG_J0)
            assert np.array_equal(g, J0[s].numpy()), f"level {s} image"
            np.testing.assert_allclose(d.debug_level(s, _lib.DIS_DBG_UINIT), r.u_init.numpy(), atol=1e-9)
            np.testing.assert_allclose(d.debug_level(s, _lib.DIS_DBG_UPATCH), r.search.u.numpy(), atol=1e-8)
            np.testing.assert_allclose(d.debug_level(s, _lib.DIS_DBG_UDENSE), r.U_dense.numpy(), atol=1e-8)
            np.testing.assert_allclose(d.debug_level(s, _lib.DIS_DBG_UREFINED), r.U_refined.numpy(), atol=1e-8)
    finally:
        d.close()


def test_identical_frames_give_exactly_zero():
    say("[zero] identical frames 1024x436")
    pr = pair("layered", 1024, 436, 100.0, 2)
    for preset in (102, 105):
        U = gpu_flow(pr.I0, pr.I0.copy(), params(preset))
        assert np.count_nonzero(U) == 0


def test_deterministic_and_graph_equals_eager():
    say("[determinism] c2b 1024x436, graph and eager")
    pr = pair("layered", 1024, 436, 100.0, 2)
    p = params(103)
    a = gpu_flow(pr.I0, pr.I1, p)
    b = gpu_flow(pr.I0, pr.I1, p)
    c = gpu_flow(pr.I0, pr.I1, params(103, flags=_lib.DIS_FLAG_NO_GRAPH))
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)


def test_pitched_frames_and_reused_handle():
    say("[pitch] 256x192 inside 300-wide rows; handle reuse across sizes")
    pr = pair("bump", 256, 192, 8.0, 1)
    p = params(101)
    ref = gpu_flow(pr.I0, pr.I1, p)
    d = DIS(p, 320, 240)
    try:
        big0 = torch.zeros(192, 300, device="cuda")
        big1 = torch.zeros(192, 300, device="cuda")
        big0[:, :256] = torch.from_numpy(pr.I0).cuda()
        big1[:, :256] = torch.from_numpy(pr.I1).cuda()
        out = d.flow(big0[:, :256], big1[:, :256])
        other = pair("bump", 300, 200, 8.0, 3)
        d.flow(torch.from_numpy(other.I0).cuda(), torch.from_numpy(other.I1).cuda())
        out2 = d.flow(big0[:, :256], big1[:, :256])
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)
        assert np.array_equal(out2.cpu().numpy().astype(np.float64), ref)
    finally:
        d.close()


def test_size_errors():
    say("[errors] sizes and pointers")
    d = DIS(params(103), 256, 256)
    try:
        x = torch.zeros(300, 200, device="cuda")
        with pytest.raises(DisError) as e:
            d.flow(x, x)
        assert e.value.code == _lib.DIS_ESIZE
        y = torch.zeros(8, 8, device="cuda")       # coarsest level smaller than a patch at scale 3
        with pytest.raises(DisError) as e:
            d.flow(y, y)
        assert e.value.code == _lib.DIS_ESIZE
        with pytest.raises(DisError) as e:
            _lib.dis_compute_flow(d.handle, 0, 0, 16, 16, 16, 0)
        assert e.value.code == _lib.DIS_EINVAL
    finally:
        d.close()


def test_lean_tiles_on_large_scales_are_bitwise_invariant():
    """A scale large enough for the lean twins of launch-mode bit 6 (the
    1024x436 pair refined at full resolution: 896 tiles of 32x16): the lean
    tiles, alone or only where a scale fills every CU twice, give the bits of
    the tiles that keep U in LDS."""
    say("[tunables] lean tiles, 1024x436 refined at scale 0")
    pr, p = pair("layered", 1024, 436, 100.0, 2), params(103, finest_scale=0)
    d = DIS(p, 1024, 436)
    try:
        t0 = torch.from_numpy(pr.I0).cuda()
        t1 = torch.from_numpy(pr.I1).cuda()
        outs = []
        for tile, mode in ((6, 1), (6, 65), (11, 1), (5, 1), (5, 65), (12, 9), (6, 73)):
            d.set_tunables(None, tile, mode)
            o = d.flow(t0, t1)
            torch.cuda.synchronize()
            outs.append(o.cpu().numpy())
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])
    finally:
        d.close()


@pytest.mark.parametrize("case", ["c2b", "c1", "inner7", "l1", "stereo", "fb", "colour"])
def test_launch_choices_are_bitwise_invariant(case):
    """Persistent vs per-phase launches, lanes per patch and refinement tiles
    change the schedule, never a bit of the flow."""
    say(f"[tunables] case {case}")
    if case == "c2b":
        pr, p = pair("layered", 1024, 436, 100.0, 2), params(103)
    elif case == "c1":
        pr, p = pair("bump", 256, 192, 8.0, 1), params(101)
    elif case == "l1":
        pr, p = pair("bump", 256, 192, 8.0, 1), params(101, norm=1)
    elif case == "stereo":
        pr, p = pair("hbump", 256, 192, 8.0, 17), params(101, flags=0x20)
    elif case == "fb":
        pr, p = pair("bump", 256, 192, 8.0, 1), params(101, flags=0x40)
    elif case == "colour":
        pr, p = pair("cbump", 288, 216, 10.0, 36), params(105, flags=0x80, var_inner=7)
    else:   # 7 SOR sweeps: each fixed-point step spans two launches
        pr, p = pair("bump", 288, 216, 10.0, 13), params(105, var_inner=7)
    h, w = pr.I0.shape[-2:]
    d = DIS(p, w, h)
    try:
        t0 = torch.from_numpy(pr.I0).cuda()
        t1 = torch.from_numpy(pr.I1).cuda()
        outs = []
        choices = [(None, 0, 0), ([4] * 16, 0, 0), ([8] * 16, 0, 0), (None, 0, 1)]
        # the persistent launch on its 16x16 tile
        choices += [(None, 1, 0), ([16] * 16, 1, 0)]
        # 32 and 64 lanes per patch (the reduction tree crosses rows of the wave)
        choices += [([32] * 16, 0, 1), ([64] * 16, 7, 1), ([64] * 16, 0, 0)]
        # every refinement tile shape / block size, with varied lanes per patch
        choices += [([[4, 8, 16][t % 3]] * 16, t, 1) for t in range(1, N_TILES)]
        # with the single-workgroup scales (launch mode bit 1)
        choices += [(None, 0, 3), (None, 3, 3), (None, 0, 2), (None, 7, 19), (None, 0, 18)]
        # without the linearisation cache (launch mode bit 3)
        choices += [(None, 7, 9), (None, 0, 8), (None, 2, 11)]
        # lean twins of the 32x16 and 16x16 tiles on the larger scales (launch mode bit 6)
        choices += [(None, 6, 65), (None, 5, 73)]
        for lpp, tile, mode in choices:
            d.set_tunables(lpp, tile, mode)
            o = d.flow(t0, t1)
            torch.cuda.synchronize()
            assert d.debug_level(0, _lib.DIS_DBG_WAIT_ERRORS) == 0
            outs.append(o.cpu().numpy())
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])
    finally:
        d.close()


FB_CASES = [
    # name, generator, preset, overrides (finest scale 0: both directions at full resolution)
    ("fb_bump_256x192", ("bump", 256, 192, 8.0, 1), 101, dict(finest_scale=0)),
    ("fb_layered_320x240", ("layered", 320, 240, 30.0, 21), 103, dict(coarsest_scale=3, finest_scale=0)),
    ("fb_norefine_raw_203x149", ("layered", 203, 149, 20.0, 22), 103,
     dict(coarsest_scale=3, finest_scale=0, refine=0, flags=0x8)),
    # stride 1: more than 32 covering patches of the other direction per pixel
    ("fb_dense_96x64", ("bump", 96, 64, 4.0, 23), 101, dict(overlap=0.875, coarsest_scale=1, finest_scale=0)),
]


@pytest.mark.parametrize("name,gen,preset,over", FB_CASES, ids=[c[0] for c in FB_CASES])
def test_fb_consistency_parity(name, gen, preset, over):
    """Forward-backward consistent densification (App. B ii): both
    directions' flows against the oracle's two-direction driver."""
    say(f"[fb] case {name}")
    from oracle import dis_oracle as O
    pr = pair(*gen)
    p = params(preset, **over)
    p.flags = int(p.flags) | _lib.DIS_FLAG_FB_CONSISTENCY
    op = oracle_params(p)
    Uf_ref, Ub_ref = (t.numpy() for t in O.dis_flow_fb(torch.from_numpy(pr.I0), torch.from_numpy(pr.I1), op))
    Uf, d = gpu_flow(pr.I0, pr.I1, p, keep=True)
    try:
        Ub = d.debug_level(0, _lib.DIS_DBG_UREFINED_BWD)
    finally:
        d.close()
    for tag, U, R, gt in (("forward", Uf, Uf_ref, pr.flow), ("backward", Ub, Ub_ref, None)):
        dd = np.sqrt(((U - R) ** 2).sum(0))
        frac = float((dd <= 1e-2).mean())
        say(f"[fb] {name} {tag}: within 1e-2 px {frac:.6f}, max diff {dd.max():.2e}")
        assert frac >= PARITY_FRAC
        if gt is not None:
            _, erel, _ = parity(U, R, gt)
            assert erel <= PARITY_EPE_REL


def test_fb_differs_from_plain_and_refusals():
    """With the merge on, the flow differs from the plain forward run, and
    the batched and backward calls refuse the merged handle."""
    say("[fb] c1 bump 256x192 plain vs merged; refusals")
    pr = pair("bump", 256, 192, 8.0, 1)
    plain = gpu_flow(pr.I0, pr.I1, params(101))
    p = params(101, flags=_lib.DIS_FLAG_FB_CONSISTENCY)
    merged, d = gpu_flow(pr.I0, pr.I1, p, keep=True)
    try:
        assert not np.array_equal(plain, merged)
        t0 = torch.from_numpy(pr.I0).cuda()
        with pytest.raises(DisError) as e:
            d.flow_batched([t0], [t0])
        assert e.value.code == _lib.DIS_EINVAL
    finally:
        d.close()
    d = DIS(params(101, flags=_lib.DIS_FLAG_FB_CONSISTENCY | _lib.DIS_FLAG_KEEP_FOR_BACKWARD), 256, 192)
    try:
        t0 = torch.from_numpy(pr.I0).cuda()
        t1 = torch.from_numpy(pr.I1).cuda()
        out = d.flow(t0, t1)
        with pytest.raises(DisError) as e:
            d.backward(torch.ones_like(out))
        assert e.value.code == _lib.DIS_EINVAL
    finally:
        d.close()


def test_colour_refusals_and_padded_rows():
    """Colour frames: padded rows (channel stride = height x pitch) give the
    same flow as packed ones; batched and backward calls refuse them."""
    say("[colour] 256x192 padded rows, refusals")
    pr = pair("cbump", 256, 192, 8.0, 31)
    p = params(101, flags=_lib.DIS_FLAG_COLOUR)
    ref = gpu_flow(pr.I0, pr.I1, p)
    d = DIS(p, 256, 192)
    try:
        b0 = torch.zeros(3, 192, 300, device="cuda")
        b1 = torch.zeros(3, 192, 300, device="cuda")
        b0[:, :, :256] = torch.from_numpy(pr.I0).cuda()
        b1[:, :, :256] = torch.from_numpy(pr.I1).cuda()
        out = d.flow(b0[:, :, :256], b1[:, :, :256])
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)
        with pytest.raises(DisError) as e:
            d.flow_batched([b0[:, :, :256]], [b1[:, :, :256]])
        assert e.value.code == _lib.DIS_EINVAL
    finally:
        d.close()
    with pytest.raises(DisError) as e:
        DIS(params(101, flags=_lib.DIS_FLAG_COLOUR | _lib.DIS_FLAG_FB_CONSISTENCY), 256, 192)
    assert e.value.code == _lib.DIS_EINVAL
    with pytest.raises(DisError) as e:
        DIS(params(101, flags=_lib.DIS_FLAG_COLOUR, patch_size=14), 256, 192)
    assert e.value.code == _lib.DIS_EINVAL
    d = DIS(params(101, flags=_lib.DIS_FLAG_COLOUR | _lib.DIS_FLAG_KEEP_FOR_BACKWARD), 256, 192)
    try:
        out = d.flow(torch.from_numpy(pr.I0).cuda(), torch.from_numpy(pr.I1).cuda())
        with pytest.raises(DisError) as e:
            d.backward(torch.ones_like(out))
        assert e.value.code == _lib.DIS_EINVAL
    finally:
        d.close()


def test_high_quality_c3a_full_size_parity():
    """The high-quality configuration at full size (1024x436, motion up to
    200 px, patch 12, overlap 0.75, 128 GN iterations, scales 4..0): the
    long Gauss-Newton chains amplify rounding the most.  The oracle takes
    about half a minute here."""
    say("[parity] case c3a_layered_1024x436_full (oracle ~30-50 s)")
    pr = pair("layered", 1024, 436, 200.0, 3)
    p = params(104)
    U_ref, _ = oracle_flow("c3a_full", pr.I0, pr.I1, oracle_params(p),
                           progress=lambda m: say(f"[parity] c3a oracle: {m}"))
    U = gpu_flow(pr.I0, pr.I1, p)
    frac, erel, dmax = parity(U, U_ref, pr.flow)
    say(f"[parity] c3a full: within 1e-2 px {frac:.6f}, mean EPE rel diff {erel:.2e}, max diff {dmax:.2e}")
    assert frac >= PARITY_FRAC
    assert erel <= PARITY_EPE_REL


def test_high_quality_c3b_full_size_parity():
    """The high-quality configuration on the large frame size (2048x1024,
    motion up to 200 px, patch 12, overlap 0.75, 128 GN iterations, scales
    4..0): 230,520 patches on the finest scale.  The oracle takes a few
    minutes here."""
    say("[parity] case c3b_layered_2048x1024_full (oracle a few minutes)")
    pr = pair("layered", 2048, 1024, 200.0, 4)
    p = params(104)
    U_ref, _ = oracle_flow("c3b_full", pr.I0, pr.I1, oracle_params(p),
                           progress=lambda m: say(f"[parity] c3b oracle: {m}"))
    say("[parity] c3b full: oracle done")
    U = gpu_flow(pr.I0, pr.I1, p)
    frac, erel, dmax = parity(U, U_ref, pr.flow)
    say(f"[parity] c3b full: within 1e-2 px {frac:.6f}, mean EPE rel diff {erel:.2e}, max diff {dmax:.2e}")
    assert frac >= PARITY_FRAC
    assert erel <= PARITY_EPE_REL


def test_large_frames_properties():
    """Frames far larger than the oracle can follow: identical 3840x2160 frames
    give exactly zero flow; an integer translation of a 1920x1080 texture is
    recovered in the interior when the finest scale is 0, and the 64
    lanes-per-patch and 16 lanes-per-patch searches agree bit for bit at this
    size."""
    say("[large] 3840x2160 identical frames; 1920x1080 translation (7, -3)")
    from paper_1603_03590_amd import synth
    rng = np.random.default_rng(77)
    tex = synth.texture(2160 + 16, 3840 + 16, rng).astype(np.float32)
    I = tex[8:8 + 2160, 8:8 + 3840].copy()
    U = gpu_flow(I, I.copy(), params(102))
    assert np.count_nonzero(U) == 0
    t = (7, -3)
    A = tex[8:8 + 1080, 8:8 + 1920].copy()
    B = tex[8 - t[1]:8 - t[1] + 1080, 8 - t[0]:8 - t[0] + 1920].copy()   # B(x + t) = A(x)
    d = DIS(params(102, finest_scale=0), 1920, 1080)
    try:
        a = torch.from_numpy(A).cuda()
        b = torch.from_numpy(B).cuda()
        outs = []
        for lanes in (16, 64):
            d.set_tunables([lanes] * 16, 7, 1)
            outs.append(d.flow(a, b).cpu().numpy().astype(np.float64))
        torch.cuda.synchronize()
    finally:
        d.close()
    assert np.array_equal(outs[0], outs[1])
    inner = outs[0][:, 64:-64, 64:-64]
    epe = np.sqrt((inner[0] - t[0]) ** 2 + (inner[1] - t[1]) ** 2)
    say(f"[large] translation: interior mean EPE {epe.mean():.3e}, 99th percentile {np.percentile(epe, 99):.3e}")
    assert epe.mean() < 1e-3          # the oracle, on a 480x272 crop of the same construction: 7e-6 px
