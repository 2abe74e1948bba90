"""Launch choices never change the flow, on random frame sizes.

Every refinement tile, the persistent and phase-major launches, the
single-workgroup scales, the linearisation cache switch and several lane
counts must give the same bits as each other (the oracle comparison is the
parity tests' job; this one covers ragged geometry: odd sizes, frames barely
larger than the patch at the finest scale, split fixed-point steps).
Every case prints itself before it touches the device.
"""
import sys

import numpy as np
import pytest
import torch

from paper_1603_03590_amd import DIS, DisError, params, synth

pytestmark = pytest.mark.gpu

# (lanes per patch or None = automatic, refinement tile, launch mode)
CHOICES = [(None, t, 1) for t in range(13)] + [
    (None, 7, 3), (None, 10, 3), (None, 10, 19), (None, 7, 0), ([16] * 16, 10, 3), ([32] * 16, 7, 3),
    (None, 10, 11), (None, 6, 65), (None, 5, 67), (None, 1, 0), ([8] * 16, 1, 0)]


def cases(n=16, seed=7):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        w, h = int(rng.integers(24, 700)), int(rng.integers(24, 400))
        preset = int(rng.choice([102, 103, 105]))
        vi = int(rng.choice([5, 5, 7, 3]))
        ps = int(rng.choice([8, 8, 12, 6]))
        sf = int(rng.integers(0, 3))
        if (w >> sf) < ps or (h >> sf) < ps:
            continue   # refused sizes are the ABI tests' business
        out.append((len(out), w, h, preset, vi, ps, sf))
    return out


@pytest.mark.parametrize("case", cases(), ids=lambda c: f"c{c[0]}_{c[1]}x{c[2]}_ps{c[5]}_vi{c[4]}_sf{c[6]}")
def test_launch_choices_bitwise_equal(case):
    k, w, h, preset, vi, ps, sf = case
    print(f"[sweep] case {k}: {w}x{h} preset {preset} patch {ps} var_inner {vi} finest {sf}", flush=True)
    sys.stdout.flush()
    pr = synth.layered_pair(w, h, 20.0, 100 + k) if k % 2 else synth.smooth_bump_pair(w, h, 8.0, 100 + k)
    d = DIS(params(preset, var_inner=vi, patch_size=ps, finest_scale=sf), w, h)
    try:
        I0 = torch.from_numpy(pr.I0).to(d.dtype).cuda()
        I1 = torch.from_numpy(pr.I1).to(d.dtype).cuda()
        ref, ran = None, 0
        for lanes, tile, mode in CHOICES:
            try:
                d.set_tunables(lanes, tile, mode)
            except DisError:
                continue   # a lane count not compiled for this patch size
            out = d.flow(I0, I1).cpu().numpy()
            ran += 1
            if ref is None:
                ref = out
            else:
                assert np.array_equal(out, ref), (tile, mode, lanes and lanes[0], float(np.abs(out - ref).max()))
        assert ran >= len(CHOICES) - 2
    finally:
        d.close()
