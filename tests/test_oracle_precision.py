"""Why the GPU path computes in float64: the oracle run in float32 misses the
parity bar (99.9% of pixels within 1e-2 px of the float64 oracle) on the
1024x436 layered workload, while a float64 run perturbed at the 1e-10 level
stays far inside it.  The method's amplifiers (weakly textured patches, the
densification weights of Eq. (3), the robust refinement weights with
eps = 1e-3 of Sec. 2.3, the 8x upscaling) turn float32 rounding into
hundredths of a pixel."""
import numpy as np
import pytest
import torch

from oracle import dis_oracle as O
from paper_1603_03590_amd import synth


def _c2a():
    # the 1024x436 workload: patch 8, overlap 0.3, scales 5..3, 12 iterations,
    # theta_vo = s + 1, theta_vi 5, refinement on
    return O.OracleParams(patch_size=8, overlap=0.3, coarsest_scale=5, finest_scale=3, gn_iters=12,
                          var_outer=-1, var_inner=5)


def _within(a, b, tol=1e-2):
    d = torch.sqrt(((a.double() - b.double()) ** 2).sum(0))
    return float((d <= tol).double().mean()), float(d.max())


@pytest.fixture(scope="module")
def c2a_pair():
    pr = synth.layered_pair(1024, 436, 100.0, 2)
    return torch.from_numpy(pr.I0), torch.from_numpy(pr.I1)


def test_float32_misses_the_parity_bar_on_the_headline_pair(c2a_pair):
    I0, I1 = c2a_pair
    p = _c2a()
    U64 = O.dis_flow(I0, I1, p)
    U32 = O.dis_flow(I0, I1, O.with_params(p, dtype=torch.float32))
    assert U32.dtype == torch.float32 and U64.dtype == torch.float64
    frac, dmax = _within(U32, U64)
    print(f"float32 oracle vs float64: {100 * frac:.2f}% of pixels within 1e-2 px, max {dmax:.3f} px")
    assert frac < 0.999


def test_float64_rounding_level_perturbation_stays_inside_the_bar(c2a_pair):
    I0, I1 = c2a_pair
    p = _c2a()
    U = O.dis_flow(I0, I1, p)
    rng = np.random.default_rng(5)
    e = torch.from_numpy(rng.standard_normal(I1.shape)) * 1e-10
    Up = O.dis_flow(I0.double(), I1.double() * (1.0 + e), p)
    frac, dmax = _within(Up, U)
    print(f"1e-10 relative perturbation: {100 * frac:.3f}% within 1e-2 px, max {dmax:.2e} px")
    assert frac == 1.0 and dmax < 1e-3
