"""FP64 CPU oracle for Dense Inverse Search optical flow (Kroeger, Timofte, Dai,
Van Gool, "Fast Optical Flow using Dense Inverse Search", ECCV 2016).

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference the GPU
path is checked against.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the HIP kernels or their host library.

Everything runs in torch float64 on the CPU, vectorised over patches and
pixels, and stays differentiable, so ``torch.autograd`` on ``dis_flow`` gives
the reference gradient with respect to both frames.

Where the paper is silent or ambiguous, a named reading fixes the step; each
reading is an attribute of ``OracleParams`` so that a test can flip it:

R1  intensities are scaled to 0..255 before anything else (the weight
    1/max(1,|d|) of Eq. (3) and the +0.01 of the data-term normalisers only
    make sense on an 8-bit scale);
R2  pyramid level s+1 is the 2x2 box mean of level s, sizes floored (Sec. 3.1,
    downscaling quotient theta_sd = 2; the filter is unstated);
R3  automatic coarsest scale ceil(log2(2 W / (f theta_ps))) with f = 8
    (Sec. 3.1), then lowered until the coarsest level is at least theta_ps
    on both sides;
R4  the template gradient (Suppl. A, S' = grad T) is the 3x3 Sobel operator
    divided by 8, replicating the border;
R5  grid stride = max(1, floor(theta_ps (1 - theta_ov))) (Sec. 2.2 step 1;
    the patch count given for the 1/8-scale Sintel level in Suppl. C needs the
    stride, not the overlap, to be floored);
R6  patches lie inside the image, top-left corners at 0, st, 2 st, ... plus a
    flush last patch at W - theta_ps (every pixel covered);
R7  patch initialisation u_init = 2 * U_{s+1}(c / 2) at the patch centre
    c = corner + (theta_ps - 1)/2 (Sec. 2.2 step 2);
R8  bilinear sampling with pixel values at integer coordinates and indices
    clamped to the image;
R9  template and warped patch are mean-normalised (Sec. 2.1); H is the sum of
    S'^T S' over the patch (Suppl. A);
R10 H is regularised as H + 1e-3 I (the paper does not treat singular H);
R11 exactly theta_it Gauss-Newton iterations, no early exit;
R12 reset to u_init when |u - u_init|_2 > theta_ps (Sec. 2.2 step 4);
R13 the densification residual d_i(x) is the mean-normalised difference at
    the final u_i (Eq. (3));
R14 densification sums over patches in ascending patch index;
R15 the refinement energy (Sec. 2.3) is linearised once per level around
    U_s; spatial derivatives are central differences [-1 0 1]/2 with
    replicated borders on the average of I0 and the warped I1;
R16 each fixed-point iteration freezes the robust weights, then runs
    theta_vi red-black SOR sweeps (red: x+y even, first; omega = 1.6); the
    smoothness weight of pixel p sits on its right and lower edges.
R17 robust error norms (App. B iii, an extension): in every Gauss-Newton
    iteration each pixel's mean-normalised residual e becomes
    sign(e) sqrt|e| (L1) or, when |e| >= b, sign(e) sqrt(2 b |e| - b^2)
    (Huber; the printed condition "e < b" is read as |e| < b, the only
    reading under which the transform is odd like the other one); the
    threshold b is not given and defaults to 1 on the 0..255 scale, the
    inlier bound of Eq. (3); the densification keeps the plain residual.
R18 stereo (App. I, an extension): the vertical degree of freedom is
    removed everywhere -- the search solves the 1-D least-squares step
    du = sum S'_x r / (H'_xx + lambda) and keeps v = 0, and the refinement
    relaxes du only (dv stays 0), so the flow's second plane is zero.
R19 forward-backward consistency (App. B ii, an extension): see
    merged_densify below for the reading of the merged Eq. (3).
R20 colour (App. B i, an extension): see colour_search below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Callable, Optional

import torch

F64 = torch.float64


@dataclass
class OracleParams:
    """Method parameters (Table 1 and Sec. 3.1) plus the reading switches."""
    patch_size: int = 8            # theta_ps
    overlap: float = 0.4           # theta_ov in [0, 1)
    coarsest_scale: int = -1       # theta_ss, -1 = automatic rule (R3)
    finest_scale: int = 3          # theta_sf
    gn_iters: int = 12             # theta_it
    var_outer: int = -1            # theta_vo, -1 = s + 1 (Sec. 3.1)
    var_inner: int = 5             # theta_vi
    delta: float = 5.0             # intensity weight
    gamma: float = 10.0            # gradient weight
    alpha: float = 10.0            # smoothness weight
    sor_omega: float = 1.6
    refine: bool = True
    # readings
    intensity_scale: float = 255.0     # R1
    auto_f: float = 8.0                # R3
    hessian_lambda: float = 1e-3       # R10
    residual: str = "normalised"       # R13: "normalised" | "raw"
    init_map: str = "literal"          # R7: "literal" x/2 | "pixel_centre" (x+0.5)/2-0.5
    grid: str = "inside"               # R6: "inside" | "overhang" (count only)
    norm: str = "l2"                   # R17: "l2" | "l1" | "huber"
    huber_b: float = 1.0               # R17
    stereo: bool = False               # R18: horizontal displacement only
    eps: float = 1e-3                  # robust penaliser epsilon (Sec. 2.3)
    # arithmetic type of the plain method (dis_flow): float64, unless a test
    # measures how far a narrower type moves the result
    dtype: torch.dtype = torch.float64


# ---------------------------------------------------------------- pyramid ----

def level_sizes(w: int, h: int, top: int):
    """[(W_s, H_s)] for s = 0..top with floored halving (R2)."""
    out = [(w, h)]
    for _ in range(top):
        w, h = w // 2, h // 2
        out.append((w, h))
    return out


def downsample2(J: torch.Tensor) -> torch.Tensor:
    """Level s+1 from level s: mean of each 2x2 block, sizes floored (R2)."""
    h2, w2 = J.shape[0] // 2, J.shape[1] // 2
    a = J[0:2 * h2:2, 0:2 * w2:2]
    b = J[0:2 * h2:2, 1:2 * w2:2]
    c = J[1:2 * h2:2, 0:2 * w2:2]
    d = J[1:2 * h2:2, 1:2 * w2:2]
    return 0.25 * (a + b + c + d)


def build_pyramid(J: torch.Tensor, top: int):
    levels = [J]
    for _ in range(top):
        levels.append(downsample2(levels[-1]))
    return levels


def auto_coarsest_scale(w: int, ps: int, f: float = 8.0) -> int:
    """Sec. 3.1: theta_ss = log2(2 w / (f theta_ps)) raised to the next
    integer, so that motions of w/f are within reach (R3 fixes f = 8)."""
    s = 0
    while (2 ** s) * f * ps < 2 * w:      # smallest s with 2^s >= 2w/(f ps)
        s += 1
    return s


def coarsest_scale(w: int, h: int, p: OracleParams) -> int:
    """theta_ss: the given value or the automatic rule, then lowered until
    the coarsest level is at least theta_ps on both sides (R3)."""
    ps = p.patch_size
    s = p.coarsest_scale if p.coarsest_scale >= 0 else auto_coarsest_scale(w, ps, p.auto_f)
    while s > 0:
        ws, hs = level_sizes(w, h, s)[-1]
        if min(ws, hs) >= ps:
            break
        s -= 1
    return s


# ---------------------------------------------------------------- helpers ----

def clamp_index(i: torch.Tensor, n: int) -> torch.Tensor:
    return i.clamp(0, n - 1)


def bilinear(img: torch.Tensor, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Bilinear interpolation of ``img`` at real coordinates (x, y) (R8).

    Pixel (row r, column c) holds the value at (x=c, y=r); the four taps are
    floor(x), floor(x)+1 (and the same in y), each clamped into the image.
    """
    h, w = img.shape
    xf = torch.floor(x)
    yf = torch.floor(y)
    ax = x - xf
    ay = y - yf
    xi = xf.long()
    yi = yf.long()
    x0 = clamp_index(xi, w)
    x1 = clamp_index(xi + 1, w)
    y0 = clamp_index(yi, h)
    y1 = clamp_index(yi + 1, h)
    top = (1 - ax) * img[y0, x0] + ax * img[y0, x1]
    bot = (1 - ax) * img[y1, x0] + ax * img[y1, x1]
    return (1 - ay) * top + ay * bot


def sobel8(J: torch.Tensor):
    """Template gradients (R4): Sobel / 8 with replicated border."""
    h, w = J.shape
    xm = clamp_index(torch.arange(w) - 1, w)
    xp = clamp_index(torch.arange(w) + 1, w)
    ym = clamp_index(torch.arange(h) - 1, h)
    yp = clamp_index(torch.arange(h) + 1, h)
    dx = J[:, xp] - J[:, xm]                    # horizontal difference per row
    gx = (dx[ym, :] + 2.0 * dx + dx[yp, :]) / 8.0
    dy = J[yp, :] - J[ym, :]
    gy = (dy[:, xm] + 2.0 * dy + dy[:, xp]) / 8.0
    return gx, gy


def grid_stride(p: OracleParams) -> int:
    """R5: the stride between patch corners."""
    return max(1, int(math.floor(p.patch_size * (1.0 - p.overlap))))


def grid_axis(n: int, ps: int, st: int, mode: str = "inside"):
    """Patch corner coordinates along one axis (R6)."""
    if mode == "overhang":
        return list(range(0, st * int(math.ceil(n / st)), st))
    pos = list(range(0, n - ps + 1, st))
    if pos[-1] != n - ps:
        pos.append(n - ps)
    return pos


def patch_grid(w: int, h: int, p: OracleParams):
    """Corners (x0, y0) of all patches, row-major (Sec. 2.2 step 1)."""
    st = grid_stride(p)
    xs = grid_axis(w, p.patch_size, st, p.grid)
    ys = grid_axis(h, p.patch_size, st, p.grid)
    x0 = torch.tensor([x for _ in ys for x in xs], dtype=torch.long)
    y0 = torch.tensor([y for y in ys for _ in xs], dtype=torch.long)
    return x0, y0, len(xs), len(ys)


def patch_offsets(ps: int):
    py, px = torch.meshgrid(torch.arange(ps), torch.arange(ps), indexing="ij")
    return px.reshape(-1), py.reshape(-1)


# --------------------------------------------------------- initialisation ----

def init_displacements(U_next: Optional[torch.Tensor], x0, y0, p: OracleParams):
    """Sec. 2.2 step 2 (R7): zero at the coarsest scale, else twice the coarser
    flow sampled at half the patch centre."""
    n = x0.numel()
    if U_next is None:
        return torch.zeros(n, 2, dtype=p.dtype)
    c = (p.patch_size - 1) / 2.0
    cx = x0.to(U_next.dtype) + c
    cy = y0.to(U_next.dtype) + c
    if p.init_map == "literal":
        qx, qy = cx / 2.0, cy / 2.0
    else:
        qx, qy = (cx + 0.5) / 2.0 - 0.5, (cy + 0.5) / 2.0 - 0.5
    return torch.stack([2.0 * bilinear(U_next[0], qx, qy),
                        2.0 * bilinear(U_next[1], qx, qy)], dim=1)


# --------------------------------------------------------- inverse search ----

def robust_residual(e: torch.Tensor, p: OracleParams) -> torch.Tensor:
    """App. B iii (R17): the residual whose square is the chosen penalty of e."""
    if p.norm == "l2":
        return e
    a = e.abs()
    if p.norm == "l1":
        t = torch.sqrt(a)
    elif p.norm == "huber":
        b = p.huber_b
        t = torch.where(a < b, a, torch.sqrt(torch.clamp(2.0 * b * a - b * b, min=0.0)))
    else:
        raise ValueError(f"unknown norm {p.norm}")
    return torch.sign(e) * t


@dataclass
class SearchResult:
    u: torch.Tensor            # [N, 2] after the reset test
    u_search: torch.Tensor     # [N, 2] before the reset test
    u_init: torch.Tensor       # [N, 2]
    reset: torch.Tensor        # [N] bool
    d: torch.Tensor            # [N, P] residual at the final u (R13)
    hessian: torch.Tensor      # [N, 2, 2] without the lambda term
    history: list = field(default_factory=list)  # u after each iteration


def inverse_search(J0, Gx, Gy, J1, x0, y0, u_init, p: OracleParams,
                   keep_history: bool = False, progress: Optional[Callable] = None) -> SearchResult:
    """Inverse-compositional Gauss-Newton search per patch (Sec. 2.1, Suppl. A).

    S' = grad T and H' = sum S'^T S' are fixed before the loop; each
    iteration warps I1 bilinearly at x + u, forms the mean-normalised
    residual r = I1(x+u) - T, solves H' du = sum S'^T r and composes
    u <- u - du.
    """
    ps = p.patch_size
    px, py = patch_offsets(ps)
    X = x0[:, None] + px[None, :]          # [N, P] integer pixel coordinates
    Y = y0[:, None] + py[None, :]
    T = J0[Y, X]
    Tn = T - T.mean(dim=1, keepdim=True)   # R9
    gx = Gx[Y, X]
    gy = Gy[Y, X]
    h11 = (gx * gx).sum(1)
    h12 = (gx * gy).sum(1)
    h22 = (gy * gy).sum(1)
    lam = p.hessian_lambda
    a11, a12, a22 = h11 + lam, h12, h22 + lam      # R10
    det = a11 * a22 - a12 * a12
    Xf = X.to(J0.dtype)
    Yf = Y.to(J0.dtype)

    u = u_init.clone()
    history = []
    for it in range(p.gn_iters):                     # R11
        if progress is not None and it > 0 and it % 32 == 0:
            progress(f"{it} of {p.gn_iters} iterations")
        Q = bilinear(J1, Xf + u[:, 0:1], Yf + u[:, 1:2])
        r = robust_residual((Q - Q.mean(dim=1, keepdim=True)) - Tn, p)
        b1 = (gx * r).sum(1)
        b2 = (gy * r).sum(1)
        if p.stereo:                                 # R18: one degree of freedom
            du = b1 / a11
            dv = torch.zeros_like(du)
        else:
            du = (a22 * b1 - a12 * b2) / det
            dv = (a11 * b2 - a12 * b1) / det
        u = u - torch.stack([du, dv], dim=1)
        if keep_history:
            history.append(u.detach().clone())

    moved = torch.sqrt(((u - u_init) ** 2).sum(1))
    reset = moved > ps                               # R12
    u_final = torch.where(reset[:, None], u_init, u)

    Q = bilinear(J1, Xf + u_final[:, 0:1], Yf + u_final[:, 1:2])
    if p.residual == "normalised":                   # R13
        d = (Q - Q.mean(dim=1, keepdim=True)) - Tn
    else:
        d = Q - T
    H = torch.stack([torch.stack([h11, h12], -1), torch.stack([h12, h22], -1)], -2)
    return SearchResult(u_final, u, u_init, reset, d, H, history)


# ---------------------------------------------------------- densification ----

def densify(w: int, h: int, x0, y0, u, d, p: OracleParams):
    """Eq. (3): per pixel, the average of the covering patches' displacements,
    each weighted by 1 / max(1, |d_i(x)|).  Returns U [2, h, w] and Z."""
    ps = p.patch_size
    px, py = patch_offsets(ps)
    lin = ((y0[:, None] + py[None, :]) * w + (x0[:, None] + px[None, :])).reshape(-1)
    wgt = 1.0 / torch.clamp(d.abs(), min=1.0)         # [N, P]
    num_u = torch.zeros(h * w, dtype=u.dtype).index_add(0, lin, (wgt * u[:, 0:1]).reshape(-1))
    num_v = torch.zeros(h * w, dtype=u.dtype).index_add(0, lin, (wgt * u[:, 1:2]).reshape(-1))
    Z = torch.zeros(h * w, dtype=u.dtype).index_add(0, lin, wgt.reshape(-1))
    U = torch.stack([num_u / Z, num_v / Z]).reshape(2, h, w)
    return U, Z.reshape(h, w)


# ------------------------------------------------------------- refinement ----

def central_dx(f):
    w = f.shape[1]
    i = torch.arange(w)
    return (f[:, clamp_index(i + 1, w)] - f[:, clamp_index(i - 1, w)]) / 2.0


def central_dy(f):
    h = f.shape[0]
    i = torch.arange(h)
    return (f[clamp_index(i + 1, h), :] - f[clamp_index(i - 1, h), :]) / 2.0


@dataclass
class RefineTerms:
    """Per-pixel linearisation of Sec. 2.3 at the current level (R15)."""
    Ix: torch.Tensor
    Iy: torch.Tensor
    Iz: torch.Tensor
    Ixx: torch.Tensor
    Ixy: torch.Tensor
    Iyy: torch.Tensor
    Ixz: torch.Tensor
    Iyz: torch.Tensor
    b0: torch.Tensor
    bx: torch.Tensor
    by: torch.Tensor


def refine_linearise(J0, J1, U) -> RefineTerms:
    h, w = J0.shape
    yy, xx = torch.meshgrid(torch.arange(h, dtype=J0.dtype), torch.arange(w, dtype=J0.dtype), indexing="ij")
    J1w = bilinear(J1, xx + U[0], yy + U[1])
    Ib = 0.5 * (J0 + J1w)
    Ix = central_dx(Ib)
    Iy = central_dy(Ib)
    Iz = J1w - J0
    Ixx = central_dx(Ix)
    Ixy = central_dy(Ix)
    Iyy = central_dy(Iy)
    Ixz = central_dx(J1w) - central_dx(J0)
    Iyz = central_dy(J1w) - central_dy(J0)
    # normalisations of the data terms (Sec. 2.3)
    b0 = 1.0 / (Ix * Ix + Iy * Iy + 0.01)
    bx = 1.0 / (Ixx * Ixx + Ixy * Ixy + 0.01)
    by = 1.0 / (Ixy * Ixy + Iyy * Iyy + 0.01)
    return RefineTerms(Ix, Iy, Iz, Ixx, Ixy, Iyy, Ixz, Iyz, b0, bx, by)


def data_energies(t: RefineTerms, du, dv):
    """E_I and E_G of Sec. 2.3 at increment (du, dv)."""
    ei = t.b0 * (t.Ix * du + t.Iy * dv + t.Iz) ** 2
    eg = (t.bx * (t.Ixx * du + t.Ixy * dv + t.Ixz) ** 2
          + t.by * (t.Ixy * du + t.Iyy * dv + t.Iyz) ** 2)
    return ei, eg


def forward_diff_x(f):
    """f(x+1) - f(x), zero in the last column."""
    return torch.cat([f[:, 1:] - f[:, :-1], torch.zeros_like(f[:, :1])], dim=1)


def forward_diff_y(f):
    return torch.cat([f[1:, :] - f[:-1, :], torch.zeros_like(f[:1, :])], dim=0)


def smooth_energy(uu, vv):
    """E_S per pixel from forward differences of the full flow (R16)."""
    return (forward_diff_x(uu) ** 2 + forward_diff_y(uu) ** 2
            + forward_diff_x(vv) ** 2 + forward_diff_y(vv) ** 2)


def robust(e, eps):
    """Psi(a^2) = sqrt(a^2 + eps^2) (Sec. 2.3)."""
    return torch.sqrt(e + eps * eps)


def linearised_energy(t: RefineTerms, U, du, dv, p: OracleParams):
    """Sum over pixels of delta Psi(E_I) + gamma Psi(E_G) + alpha Psi(E_S)."""
    ei, eg = data_energies(t, du, dv)
    es = smooth_energy(U[0] + du, U[1] + dv)
    return (p.delta * robust(ei, p.eps) + p.gamma * robust(eg, p.eps)
            + p.alpha * robust(es, p.eps)).sum()


@dataclass
class SorSystem:
    """The quadratic of one fixed-point iteration: per-pixel 2x2 data matrix
    A, vector b, and the smoothness weight ws owned by each pixel's right and
    lower edges."""
    A11: torch.Tensor
    A12: torch.Tensor
    A22: torch.Tensor
    b1: torch.Tensor
    b2: torch.Tensor
    ws: torch.Tensor


def sor_system(t: RefineTerms, U, du, dv, p: OracleParams) -> SorSystem:
    """Freeze the robust weights at the current increment (R16)."""
    ei, eg = data_energies(t, du, dv)
    pi = p.delta / (2.0 * robust(ei, p.eps))
    pg = p.gamma / (2.0 * robust(eg, p.eps))
    ws = p.alpha / (2.0 * robust(smooth_energy(U[0] + du, U[1] + dv), p.eps))
    A11 = pi * t.b0 * t.Ix * t.Ix + pg * (t.bx * t.Ixx * t.Ixx + t.by * t.Ixy * t.Ixy)
    A12 = pi * t.b0 * t.Ix * t.Iy + pg * (t.bx * t.Ixx * t.Ixy + t.by * t.Ixy * t.Iyy)
    A22 = pi * t.b0 * t.Iy * t.Iy + pg * (t.bx * t.Ixy * t.Ixy + t.by * t.Iyy * t.Iyy)
    b1 = pi * t.b0 * t.Ix * t.Iz + pg * (t.bx * t.Ixx * t.Ixz + t.by * t.Ixy * t.Iyz)
    b2 = pi * t.b0 * t.Iy * t.Iz + pg * (t.bx * t.Ixy * t.Ixz + t.by * t.Iyy * t.Iyz)
    return SorSystem(A11, A12, A22, b1, b2, ws)


def quadratic_energy(sys: SorSystem, U, du, dv):
    """The frozen-weight quadratic that the SOR sweeps decrease:
    sum du^T A du + 2 b^T du + ws * (squared forward differences of U + dU)."""
    data = (sys.A11 * du * du + 2 * sys.A12 * du * dv + sys.A22 * dv * dv
            + 2 * (sys.b1 * du + sys.b2 * dv))
    sm = sys.ws * smooth_energy(U[0] + du, U[1] + dv)
    return (data + sm).sum()


def _neighbour_sums(ws, f):
    """For each pixel p: S = sum of the weights of its edges and
    N = sum over 4-neighbours q of w_pq * f(q); edges leaving the image are
    dropped (Neumann)."""
    h, w = f.shape
    wr = torch.cat([ws[:, :-1], torch.zeros_like(ws[:, :1])], 1)     # edge p -> p+ex
    wl = torch.cat([torch.zeros_like(ws[:, :1]), ws[:, :-1]], 1)     # edge p-ex -> p
    wd = torch.cat([ws[:-1, :], torch.zeros_like(ws[:1, :])], 0)     # edge p -> p+ey
    wu = torch.cat([torch.zeros_like(ws[:1, :]), ws[:-1, :]], 0)     # edge p-ey -> p
    fr = torch.cat([f[:, 1:], torch.zeros_like(f[:, :1])], 1)
    fl = torch.cat([torch.zeros_like(f[:, :1]), f[:, :-1]], 1)
    fd = torch.cat([f[1:, :], torch.zeros_like(f[:1, :])], 0)
    fu = torch.cat([torch.zeros_like(f[:1, :]), f[:-1, :]], 0)
    S = wr + wl + wd + wu
    N = wr * fr + wl * fl + wd * fd + wu * fu
    return S, N


def sor_sweeps(sys: SorSystem, U, du, dv, n_sweeps: int, omega: float,
               on_half_sweep: Optional[Callable] = None, stereo: bool = False):
    """``n_sweeps`` red-black SOR sweeps on the frozen system (R16).

    For the pixels of one colour (all independent, their 4-neighbours have the
    other colour): du_p is relaxed first, then dv_p using the new du_p.
    """
    h, w = du.shape
    yy, xx = torch.meshgrid(torch.arange(h), torch.arange(w), indexing="ij")
    colour = (xx + yy) % 2
    Uu, Uv = U[0], U[1]
    S, NUu = _neighbour_sums(sys.ws, Uu)
    _, NUv = _neighbour_sums(sys.ws, Uv)
    for _ in range(n_sweeps):
        for c in (0, 1):
            m = colour == c
            _, Ndu = _neighbour_sums(sys.ws, du)
            num = NUu + Ndu - S * Uu - sys.b1 - sys.A12 * dv
            du_new = (1 - omega) * du + omega * num / (sys.A11 + S)
            du = torch.where(m, du_new, du)
            if not stereo:                           # R18: dv stays 0
                _, Ndv = _neighbour_sums(sys.ws, dv)
                num = NUv + Ndv - S * Uv - sys.b2 - sys.A12 * du
                dv_new = (1 - omega) * dv + omega * num / (sys.A22 + S)
                dv = torch.where(m, dv_new, dv)
            if on_half_sweep is not None:
                on_half_sweep(du, dv)
    return du, dv


def refine(J0, J1, U, n_outer: int, p: OracleParams, trace: Optional[Callable] = None):
    """Variational refinement of one level (Sec. 2.3, R15, R16).

    ``trace(kind, k, terms, system, du, dv)`` is called at the start of each
    fixed-point iteration (kind "outer") and after every half-sweep (kind
    "half"), for the energy tests.
    """
    t = refine_linearise(J0, J1, U)
    du = torch.zeros_like(U[0])
    dv = torch.zeros_like(U[1])
    for k in range(n_outer):
        sys = sor_system(t, U, du, dv, p)
        if trace is not None:
            trace("outer", k, t, sys, du, dv)
            cb = lambda a, b, k=k, sys=sys: trace("half", k, t, sys, a, b)
        else:
            cb = None
        du, dv = sor_sweeps(sys, U, du, dv, p.var_inner, p.sor_omega, cb, stereo=p.stereo)
    return torch.stack([U[0] + du, U[1] + dv])


# -------------------------------------------------------------- upsampling ---

def upsample(U: torch.Tensor, w: int, h: int, s: int, p: OracleParams) -> torch.Tensor:
    """Bilinear upscaling of the level-s flow to w x h, vectors times 2^s
    (Sec. 3.1, final paragraph)."""
    if s == 0:
        return U
    f = float(2 ** s)
    yy, xx = torch.meshgrid(torch.arange(h, dtype=U.dtype), torch.arange(w, dtype=U.dtype), indexing="ij")
    if p.init_map == "literal":
        qx, qy = xx / f, yy / f
    else:
        qx, qy = (xx + 0.5) / f - 0.5, (yy + 0.5) / f - 0.5
    return torch.stack([f * bilinear(U[0], qx, qy), f * bilinear(U[1], qx, qy)])


# ---------------------------------------------------------------- driver -----

@dataclass
class LevelRecord:
    s: int
    u_init: torch.Tensor
    search: SearchResult
    U_dense: torch.Tensor
    U_refined: torch.Tensor
    n_outer: int


def outer_iterations(s: int, p: OracleParams) -> int:
    return s + 1 if p.var_outer < 0 else p.var_outer


def dis_flow(I0: torch.Tensor, I1: torch.Tensor, p: OracleParams, records: Optional[list] = None,
             progress: Optional[Callable] = None):
    """Dense Inverse Search, Alg. 1: coarse-to-fine over s = theta_ss .. theta_sf
    of grid, initialisation, inverse search, densification and refinement,
    then upscaling to the input resolution.  Returns the flow [2, H, W].
    `progress`, if given, receives a line of text as the work advances (long
    runs); it takes no part in the computation."""
    I0 = torch.as_tensor(I0).to(p.dtype)
    I1 = torch.as_tensor(I1).to(p.dtype)
    h, w = I0.shape
    ss = coarsest_scale(w, h, p)
    sf = p.finest_scale
    if sf > ss:
        raise ValueError(f"finest scale {sf} above coarsest scale {ss}")
    J0 = build_pyramid(p.intensity_scale * I0, ss)      # R1, R2
    J1 = build_pyramid(p.intensity_scale * I1, ss)
    U = None
    for s in range(ss, sf - 1, -1):
        hs, ws_ = J0[s].shape
        if min(ws_, hs) < p.patch_size:
            raise ValueError(f"level {s} ({ws_}x{hs}) smaller than the patch")
        Gx, Gy = sobel8(J0[s])
        x0, y0, _, _ = patch_grid(ws_, hs, p)
        u_init = init_displacements(U, x0, y0, p)
        tell = None if progress is None else (lambda m, s=s: progress(f"scale {s}: search, {m}"))
        res = inverse_search(J0[s], Gx, Gy, J1[s], x0, y0, u_init, p, progress=tell)
        Ud, _ = densify(ws_, hs, x0, y0, res.u, res.d, p)
        n_outer = outer_iterations(s, p)
        Ur = refine(J0[s], J1[s], Ud, n_outer, p) if p.refine else Ud
        if records is not None:
            records.append(LevelRecord(s, u_init, res, Ud, Ur, n_outer))
        if progress is not None:
            progress(f"scale {s} done ({ws_}x{hs}, {x0.numel()} patches)")
        U = Ur
    return upsample(U, w, h, sf, p)


def endpoint_error(flow, gt):
    """Per-pixel end-point error |U - U_gt|_2 (Sec. 3)."""
    return torch.sqrt(((torch.as_tensor(flow) - torch.as_tensor(gt)) ** 2).sum(0))


def with_params(p: OracleParams, **kw) -> OracleParams:
    return replace(p, **kw)


# ------------------------------------- forward-backward consistency (App. B ii)
#
# R19 (an extension): both directions run the whole method; only the
# densification merges them.  For the flow of frame A (reference) the patches
# of A's own search vote as in Eq. (3); every patch j of the other direction's
# search, found on B's grid and displaced by its u_j into A, votes -u_j at the
# pixels x of A with x - u_j inside its template square [x0_j, x0_j+ps-1]^2
# (closed, continuous), with the residual A(x) - T_j(x - u_j) (T_j sampled
# bilinearly in B), mean-normalised by that patch's mean residual at its final
# u_j (as R13), weighted 1 / max(1, |d|).  Own patches are summed first in
# ascending index, then the other direction's in ascending index.  Each
# direction is refined on its own, and the next scale initialises each
# direction from its own flow.

def patch_mean_residual(Jref, Jother, x0, y0, u, p: OracleParams):
    """Mean over the template of Jother(x + u) - Jref(x) at the patches' final u."""
    ps = p.patch_size
    px, py = patch_offsets(ps)
    X = (x0[:, None] + px[None, :]).to(F64)
    Y = (y0[:, None] + py[None, :]).to(F64)
    Q = bilinear(Jother, X + u[:, 0:1], Y + u[:, 1:2])
    T = Jref[(y0[:, None] + py[None, :]), (x0[:, None] + px[None, :])]
    return (Q - T).mean(dim=1)


def merged_densify(Jref, Jother, x0, y0, u_own, d_own, u_other, md_other, p: OracleParams,
                   merge: bool = True):
    """The densification of App. B ii for the flow of frame Jref: Eq. (3) over
    the own patches plus the other direction's displaced patches (R19); both
    directions use the same grid."""
    return merged_densify_pairs(Jref, Jother, x0, y0, u_own, d_own, x0 if merge else x0[:0],
                                y0 if merge else y0[:0], u_other if merge else u_other[:0],
                                md_other if merge else md_other[:0], p)


def merged_densify_pairs(Jref, Jother, x0, y0, u_own, d_own, xo, yo, u_other, md_other, p: OracleParams,
                         want_z: bool = False):
    """merged_densify with the other direction's patch corners (xo, yo) given
    separately; returns U [2, h, w] (or Z when want_z)."""
    h, w = Jref.shape
    ps = p.patch_size
    px, py = patch_offsets(ps)
    # own patches, ascending i
    lin = ((y0[:, None] + py[None, :]) * w + (x0[:, None] + px[None, :])).reshape(-1)
    wgt = 1.0 / torch.clamp(d_own.abs(), min=1.0)
    num_u = torch.zeros(h * w, dtype=F64).index_add(0, lin, (wgt * u_own[:, 0:1]).reshape(-1))
    num_v = torch.zeros(h * w, dtype=F64).index_add(0, lin, (wgt * u_own[:, 1:2]).reshape(-1))
    Z = torch.zeros(h * w, dtype=F64).index_add(0, lin, wgt.reshape(-1))
    # the other direction's patches, ascending j, each over the pixels of
    # Jref its displaced square covers
    if u_other.shape[0]:
        for j in range(u_other.shape[0]):
            uj, vj = float(u_other[j, 0]), float(u_other[j, 1])
            xa, xb = float(xo[j]) + uj, float(xo[j]) + ps - 1 + uj
            ya, yb = float(yo[j]) + vj, float(yo[j]) + ps - 1 + vj
            xl, xh = max(0, math.ceil(xa)), min(w - 1, math.floor(xb))
            yl, yh = max(0, math.ceil(ya)), min(h - 1, math.floor(yb))
            if xl > xh or yl > yh:      # displaced square misses the level
                continue
            cx = torch.arange(xl, xh + 1)
            cy = torch.arange(yl, yh + 1)
            YY, XX = torch.meshgrid(cy, cx, indexing="ij")
            tv = bilinear(Jother, XX.to(F64) - uj, YY.to(F64) - vj)
            d = Jref[YY, XX] - tv
            if p.residual == "normalised":
                d = d - md_other[j]
            wj = 1.0 / torch.clamp(d.abs(), min=1.0)
            li = (YY * w + XX).reshape(-1)
            num_u = num_u.index_add(0, li, (-uj * wj).reshape(-1))
            num_v = num_v.index_add(0, li, (-vj * wj).reshape(-1))
            Z = Z.index_add(0, li, wj.reshape(-1))
    if want_z:
        return Z.reshape(h, w)
    return torch.stack([num_u / Z, num_v / Z]).reshape(2, h, w)


def dis_flow_fb(I0, I1, p: OracleParams, merge: bool = True):
    """Forward and backward flow with forward-backward consistent
    densification (App. B ii, R19).  Returns (U forward [2,H,W], U backward)."""
    I0 = torch.as_tensor(I0).to(F64)
    I1 = torch.as_tensor(I1).to(F64)
    h, w = I0.shape
    ss = coarsest_scale(w, h, p)
    sf = p.finest_scale
    if sf > ss:
        raise ValueError(f"finest scale {sf} above coarsest scale {ss}")
    P0 = build_pyramid(p.intensity_scale * I0, ss)
    P1 = build_pyramid(p.intensity_scale * I1, ss)
    Uf = Ub = None
    for s in range(ss, sf - 1, -1):
        hs, ws_ = P0[s].shape
        x0, y0, _, _ = patch_grid(ws_, hs, p)
        res = []
        for Ja, Jb, Uprev in ((P0[s], P1[s], Uf), (P1[s], P0[s], Ub)):
            Gx, Gy = sobel8(Ja)
            r = inverse_search(Ja, Gx, Gy, Jb, x0, y0, init_displacements(Uprev, x0, y0, p), p)
            res.append((r, patch_mean_residual(Ja, Jb, x0, y0, r.u, p)))
        (rf, mdf), (rb, mdb) = res
        Udf = merged_densify(P0[s], P1[s], x0, y0, rf.u, rf.d, rb.u, mdb, p, merge)
        Udb = merged_densify(P1[s], P0[s], x0, y0, rb.u, rb.d, rf.u, mdf, p, merge)
        n_outer = outer_iterations(s, p)
        if p.refine:
            Uf = refine(P0[s], P1[s], Udf, n_outer, p)
            Ub = refine(P1[s], P0[s], Udb, n_outer, p)
        else:
            Uf, Ub = Udf, Udb
    return upsample(Uf, w, h, sf, p), upsample(Ub, w, h, sf, p)


# ------------------------------------------------------------ colour (App. B i)
#
# R20 (an extension): frames have C channels (RGB: 3), each scaled to 0..255
# with a pyramid of its own (R1, R2 per channel).  The search minimises the
# patch error summed over the channels: every channel is mean-normalised on
# its own (R9), S'^c is the Sobel/8 gradient of channel c of the template, and
# H' and the right-hand side are sums over channels of the grey ones (R10's
# lambda is added once); R17's transform acts on each channel's residual.  The
# densification weight of Eq. (3) takes |d_i(x)| as the Euclidean norm over
# channels of the per-channel residuals of R13 (one channel: |d|).  The
# refinement uses all channels jointly, in the multi-channel form of the
# variational method the paper cites: the brightness and gradient data terms
# are sums over channels of the grey terms, each channel with its own
# linearisation and normalisers (R15), and one robust function per term
# applied to the channel sum; the smoothness term is unchanged.

def colour_search(J0s, J1s, x0, y0, u_init, p: OracleParams) -> SearchResult:
    """Inverse search on C-channel levels ([C, h, w]); ``d`` of the result
    is [C, N, P] (the per-channel residual at the final u)."""
    ps = p.patch_size
    px, py = patch_offsets(ps)
    X = x0[:, None] + px[None, :]
    Y = y0[:, None] + py[None, :]
    C = J0s.shape[0]
    T, Tn, gx, gy = [], [], [], []
    for c in range(C):
        Gx, Gy = sobel8(J0s[c])
        T.append(J0s[c][Y, X])
        Tn.append(T[c] - T[c].mean(dim=1, keepdim=True))
        gx.append(Gx[Y, X])
        gy.append(Gy[Y, X])
    h11 = sum((gx[c] * gx[c]).sum(1) for c in range(C))
    h12 = sum((gx[c] * gy[c]).sum(1) for c in range(C))
    h22 = sum((gy[c] * gy[c]).sum(1) for c in range(C))
    lam = p.hessian_lambda
    a11, a12, a22 = h11 + lam, h12, h22 + lam
    det = a11 * a22 - a12 * a12
    Xf = X.to(F64)
    Yf = Y.to(F64)

    u = u_init.clone()
    for _ in range(p.gn_iters):
        b1 = torch.zeros_like(h11)
        b2 = torch.zeros_like(h11)
        for c in range(C):
            Q = bilinear(J1s[c], Xf + u[:, 0:1], Yf + u[:, 1:2])
            r = robust_residual((Q - Q.mean(dim=1, keepdim=True)) - Tn[c], p)
            b1 = b1 + (gx[c] * r).sum(1)
            b2 = b2 + (gy[c] * r).sum(1)
        if p.stereo:
            du = b1 / a11
            dv = torch.zeros_like(du)
        else:
            du = (a22 * b1 - a12 * b2) / det
            dv = (a11 * b2 - a12 * b1) / det
        u = u - torch.stack([du, dv], dim=1)

    moved = torch.sqrt(((u - u_init) ** 2).sum(1))
    reset = moved > ps
    u_final = torch.where(reset[:, None], u_init, u)
    d = []
    for c in range(C):
        Q = bilinear(J1s[c], Xf + u_final[:, 0:1], Yf + u_final[:, 1:2])
        d.append((Q - Q.mean(dim=1, keepdim=True)) - Tn[c] if p.residual == "normalised" else Q - T[c])
    H = torch.stack([torch.stack([h11, h12], -1), torch.stack([h12, h22], -1)], -2)
    return SearchResult(u_final, u, u_init, reset, torch.stack(d), H, [])


def colour_densify(w: int, h: int, x0, y0, u, d, p: OracleParams):
    """Eq. (3) with |d_i(x)| the norm over channels of d [C, N, P]."""
    return densify(w, h, x0, y0, u, torch.sqrt((d * d).sum(0)), p)


def colour_linearise(J0s, J1s, U):
    """R15 per channel: one RefineTerms per channel."""
    return [refine_linearise(J0s[c], J1s[c], U) for c in range(J0s.shape[0])]


def colour_data_energies(ts, du, dv):
    """Channel sums of the grey E_I and E_G at increment (du, dv)."""
    ei, eg = 0.0, 0.0
    for t in ts:
        a, b = data_energies(t, du, dv)
        ei = ei + a
        eg = eg + b
    return ei, eg


def colour_sor_system(ts, U, du, dv, p: OracleParams) -> SorSystem:
    """One robust weight per data term over the channel sum; the matrix and
    vector are channel sums of the grey ones at those weights."""
    ei, eg = colour_data_energies(ts, du, dv)
    pi = p.delta / (2.0 * robust(ei, p.eps))
    pg = p.gamma / (2.0 * robust(eg, p.eps))
    ws = p.alpha / (2.0 * robust(smooth_energy(U[0] + du, U[1] + dv), p.eps))
    A11 = A12 = A22 = b1 = b2 = 0.0
    for t in ts:
        A11 = A11 + pi * t.b0 * t.Ix * t.Ix + pg * (t.bx * t.Ixx * t.Ixx + t.by * t.Ixy * t.Ixy)
        A12 = A12 + pi * t.b0 * t.Ix * t.Iy + pg * (t.bx * t.Ixx * t.Ixy + t.by * t.Ixy * t.Iyy)
        A22 = A22 + pi * t.b0 * t.Iy * t.Iy + pg * (t.bx * t.Ixy * t.Ixy + t.by * t.Iyy * t.Iyy)
        b1 = b1 + pi * t.b0 * t.Ix * t.Iz + pg * (t.bx * t.Ixx * t.Ixz + t.by * t.Ixy * t.Iyz)
        b2 = b2 + pi * t.b0 * t.Iy * t.Iz + pg * (t.bx * t.Ixy * t.Ixz + t.by * t.Iyy * t.Iyz)
    return SorSystem(A11, A12, A22, b1, b2, ws)


def colour_refine(J0s, J1s, U, n_outer: int, p: OracleParams):
    ts = colour_linearise(J0s, J1s, U)
    du = torch.zeros_like(U[0])
    dv = torch.zeros_like(U[1])
    for _ in range(n_outer):
        sys = colour_sor_system(ts, U, du, dv, p)
        du, dv = sor_sweeps(sys, U, du, dv, p.var_inner, p.sor_omega, stereo=p.stereo)
    return torch.stack([U[0] + du, U[1] + dv])


def dis_flow_colour(I0: torch.Tensor, I1: torch.Tensor, p: OracleParams, records: Optional[list] = None):
    """Alg. 1 on C-channel frames [C, H, W] (R20).  Returns the flow [2, H, W]."""
    I0 = torch.as_tensor(I0).to(F64)
    I1 = torch.as_tensor(I1).to(F64)
    C, h, w = I0.shape
    ss = coarsest_scale(w, h, p)
    sf = p.finest_scale
    if sf > ss:
        raise ValueError(f"finest scale {sf} above coarsest scale {ss}")
    P0 = [build_pyramid(p.intensity_scale * I0[c], ss) for c in range(C)]
    P1 = [build_pyramid(p.intensity_scale * I1[c], ss) for c in range(C)]
    U = None
    for s in range(ss, sf - 1, -1):
        J0s = torch.stack([P0[c][s] for c in range(C)])
        J1s = torch.stack([P1[c][s] for c in range(C)])
        hs, ws_ = J0s.shape[1:]
        x0, y0, _, _ = patch_grid(ws_, hs, p)
        u_init = init_displacements(U, x0, y0, p)
        res = colour_search(J0s, J1s, x0, y0, u_init, p)
        Ud, _ = colour_densify(ws_, hs, x0, y0, res.u, res.d, p)
        n_outer = outer_iterations(s, p)
        Ur = colour_refine(J0s, J1s, Ud, n_outer, p) if p.refine else Ud
        if records is not None:
            records.append(LevelRecord(s, u_init, res, Ud, Ur, n_outer))
        U = Ur
    return upsample(U, w, h, sf, p)
