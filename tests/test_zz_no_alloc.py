"""The flow call without a handle (static device scratch) against the
handle-based call, through the C ABI: two calls in a row, the second on a
smaller pair, each bitwise equal to dis_compute_flow with the same
parameters (and so within the oracle-parity bar that call meets)."""
import sys

import numpy as np
import pytest
import torch

from dis_cases import pair
from paper_1603_03590_amd import DisError, params, _lib

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def handle_flow(p, t0, t1, w, h):
    """dis_compute_flow on a fresh handle sized for this pair."""
    hd = _lib.dis_create(p, w, h, 1, torch.cuda.current_stream().cuda_stream)
    try:
        out = torch.empty(2, h, w, dtype=torch.float32, device="cuda")
        _lib.dis_compute_flow(hd, t0.data_ptr(), t1.data_ptr(), w, h, t0.stride(0), out.data_ptr())
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        _lib.dis_destroy(hd)


def noalloc_flow(p, t0, t1, w, h):
    out = torch.full((2, h, w), float("nan"), dtype=torch.float32, device="cuda")
    _lib.dis_compute_flow_noalloc(p, t0.data_ptr(), t1.data_ptr(), w, h, t0.stride(0), out.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def frames(gen, pitch_pad=0):
    pr = pair(*gen)
    h, w = pr.I0.shape
    t0 = torch.zeros(h, w + pitch_pad, dtype=torch.float32, device="cuda")
    t1 = torch.zeros(h, w + pitch_pad, dtype=torch.float32, device="cuda")
    t0[:, :w] = torch.from_numpy(pr.I0).cuda()
    t1[:, :w] = torch.from_numpy(pr.I1).cuda()
    return t0, t1, w, h


# (case, generator (kind, w, h, max displacement, seed), preset, overrides, row padding)
SEQUENCES = [
    ("c2a_then_c1", [(("layered", 1024, 436, 100.0, 2), 102, {}, 0),
                     (("bump", 256, 192, 8.0, 1), 101, {}, 0)]),
    ("c3_shape_then_ragged", [(("layered", 640, 480, 60.0, 9), 104, dict(gn_iters=32, var_outer=2), 0),
                              (("layered", 203, 149, 20.0, 8), 103, dict(coarsest_scale=3, finest_scale=0), 5)]),
]


@pytest.mark.parametrize("name,calls", SEQUENCES, ids=[s[0] for s in SEQUENCES])
def test_noalloc_matches_handle_call(name, calls):
    for k, (gen, preset, over, pad) in enumerate(calls):
        say(f"[noalloc] {name} call {k}: {gen[1]}x{gen[2]} preset {preset} {over} pitch pad {pad}")
        p = params(preset, **over)
        t0, t1, w, h = frames(gen, pad)
        ref = handle_flow(p, t0, t1, w, h)
        got = noalloc_flow(p, t0, t1, w, h)
        assert np.isfinite(got).all()
        diff = np.sqrt(((got.astype(np.float64) - ref) ** 2).sum(0))
        say(f"[noalloc] {name} call {k}: max |diff| {diff.max():.3e}, equal bits {np.array_equal(got, ref)}")
        assert (diff <= 1e-2).mean() >= 0.999
        assert np.array_equal(got, ref)


def test_noalloc_rejects_what_it_cannot_hold():
    say("[noalloc] error paths (host-side checks, no kernel runs)")
    t = torch.zeros(8, 8, device="cuda")
    too_big = params(104)                      # theta_sf 0 at 4096x4096: far beyond the static scratch
    with pytest.raises(DisError) as e:
        _lib.dis_compute_flow_noalloc(too_big, t.data_ptr(), t.data_ptr(), 4096, 4096, 4096, t.data_ptr())
    assert e.value.code == _lib.DIS_ESIZE
    assert "static scratch" in _lib.dis_last_error()
    with pytest.raises(DisError) as e:
        _lib.dis_compute_flow_noalloc(params(105, flags=_lib.DIS_FLAG_KEEP_FOR_BACKWARD), t.data_ptr(),
                                      t.data_ptr(), 512, 256, 512, t.data_ptr())
    assert e.value.code == _lib.DIS_EINVAL
    with pytest.raises(DisError) as e:
        _lib.dis_compute_flow_noalloc(params(102), 0, t.data_ptr(), 1024, 436, 1024, t.data_ptr())
    assert e.value.code == _lib.DIS_EINVAL
    # a failed call leaves the next one working
    t0, t1, w, h = frames(("bump", 256, 192, 8.0, 1))
    p = params(101)
    assert np.array_equal(noalloc_flow(p, t0, t1, w, h), handle_flow(p, t0, t1, w, h))
