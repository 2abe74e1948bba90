// HIP kernels of Dense Inverse Search optical flow for gfx950 (CDNA4).
//
// All arithmetic is float64: the pipeline (search, densification weights,
// robust refinement weights, upscaling) amplifies rounding noise by up to
// ~1e6, and on CDNA4 a float64 FMA issues at the same per-lane rate as an
// unpacked float32 one.  Frames arrive as float32 and are widened exactly.
//
// Built with -ffp-contract=off: every multiply-add the kernels fuse is an
// explicit fma(), so results do not depend on template instance or launch
// shape (the search's lanes-per-patch and the refinement's tile are free to
// change without changing a bit of the output).
#include <hip/hip_runtime.h>
#include "dis_internal.h"

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// Bilinear sample, pixel values at integer coordinates, taps clamped to the
// image.  Coordinates far outside are pulled to two pixels beyond the
// border first; that leaves the clamped taps (and so the value) unchanged.
__device__ __forceinline__ double bilin(const double* __restrict__ img, int W, int H, double x, double y) {
    double xf = floor(x), yf = floor(y);
    const double ax = x - xf, ay = y - yf;
    xf = fmin(fmax(xf, -2.0), (double)W + 1.0);
    yf = fmin(fmax(yf, -2.0), (double)H + 1.0);
    const int xi = (int)xf, yi = (int)yf;
    const int x0 = clampi(xi, 0, W - 1), x1 = clampi(xi + 1, 0, W - 1);
    const int y0 = clampi(yi, 0, H - 1), y1 = clampi(yi + 1, 0, H - 1);
    const double top = (1.0 - ax) * img[y0 * W + x0] + ax * img[y0 * W + x1];
    const double bot = (1.0 - ax) * img[y1 * W + x0] + ax * img[y1 * W + x1];
    return (1.0 - ay) * top + ay * bot;
}

// ------------------------------------------------------------------ pyramid

__global__ __launch_bounds__(256) void k_pyramid(const PyrArgs a) {
    __shared__ double t0[32][33];
    __shared__ double t1[16][17];
    const int f = blockIdx.y;
    const int bx = blockIdx.x % a.tiles_x, by = blockIdx.x / a.tiles_x;
    const int X0 = bx * 32, Y0 = by * 32;
    for (int i = threadIdx.x; i < 1024; i += 256) {
        const int ly = i >> 5, lx = i & 31;
        const int x = X0 + lx, y = Y0 + ly;
        double v = 0.0;
        if (x < a.w0 && y < a.h0) {
            const size_t g = (size_t)y * a.src_pitch + x;
            if (a.src_kind == 1)
                v = a.scale * (double)((const float*)a.src[f])[g];
            else
                v = a.scale * ((const double*)a.src[f])[g];
            if (a.lvl0[f]) a.lvl0[f][(size_t)y * a.w0 + x] = v;
        }
        t0[ly][lx] = v;
    }
    __syncthreads();
    int n = 32;
    for (int k = 1; k <= a.nlev; ++k) {
        n >>= 1;
        // level k of the tile (n x n <= 256, one pixel per thread): mean of a
        // 2x2 block of level k-1, summed row-major ((a+b)+c)+d, then scaled
        const bool from0 = (k & 1);
        const bool act = threadIdx.x < n * n;
        const int ly = threadIdx.x / n, lx = threadIdx.x - ly * n;
        double v = 0.0;
        if (act) {
            if (from0)
                v = 0.25 * (((t0[2 * ly][2 * lx] + t0[2 * ly][2 * lx + 1]) + t0[2 * ly + 1][2 * lx]) +
                            t0[2 * ly + 1][2 * lx + 1]);
            else
                v = 0.25 * (((t1[2 * ly][2 * lx] + t1[2 * ly][2 * lx + 1]) + t1[2 * ly + 1][2 * lx]) +
                            t1[2 * ly + 1][2 * lx + 1]);
            const int xs = (X0 >> k) + lx, ys = (Y0 >> k) + ly;
            double* d = a.dst[f][k];
            if (d && xs < a.ws[k] && ys < a.hs[k]) d[(size_t)ys * a.ws[k] + xs] = v;
        }
        __syncthreads();   // every read of the source buffer precedes the overwrite
        if (act) {
            if (from0) t1[ly][lx] = v; else t0[ly][lx] = v;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ search

// Canonical patch sums.  A patch's pixels p = 0..PS*PS-1 form 16 groups of
// GS = ceil(PS*PS/16) consecutive pixels; a group is summed sequentially
// (fma for products), then the 16 group sums pairwise in a fixed binary tree.
// A lane holds GPL = 16/LPP consecutive groups; the tree levels inside a lane
// are done in registers, the rest by xor shuffles across the LPP lanes of
// the patch.  The order is the same for every LPP.
template <int GS, int GPL, int LPP>
__device__ __forceinline__ double tree_finish(double (&g)[GPL]) {
#pragma unroll
    for (int step = 1; step < GPL; step <<= 1)
#pragma unroll
        for (int j = 0; j < GPL; j += 2 * step) g[j] = g[j] + g[j + step];
    double s = g[0];
#pragma unroll
    for (int off = 1; off < LPP; off <<= 1) s = s + __shfl_xor(s, off, 64);
    return s;
}

template <int GS, int GPL, int LPP>
__device__ __forceinline__ double csum(const double (&v)[GS * GPL]) {
    double g[GPL];
#pragma unroll
    for (int j = 0; j < GPL; ++j) {
        double s = v[j * GS];
#pragma unroll
        for (int k = 1; k < GS; ++k) s = s + v[j * GS + k];
        g[j] = s;
    }
    return tree_finish<GS, GPL, LPP>(g);
}

template <int GS, int GPL, int LPP>
__device__ __forceinline__ double csum_prod(const double (&a)[GS * GPL], const double (&b)[GS * GPL]) {
    double g[GPL];
#pragma unroll
    for (int j = 0; j < GPL; ++j) {
        double s = a[j * GS] * b[j * GS];
#pragma unroll
        for (int k = 1; k < GS; ++k) s = fma(a[j * GS + k], b[j * GS + k], s);
        g[j] = s;
    }
    return tree_finish<GS, GPL, LPP>(g);
}

// One thread group of LPP lanes per patch, 256 threads per block.  Patch
// corners, initialisation (Sec. 2.2 steps 1-2), template and Sobel/8
// gradients, the precomputed 2x2 Hessian, theta_it inverse-compositional
// updates u <- u - H^-1 sum grad(T) r (Suppl. A), the reset test of step 4,
// and the mean residual at the final u, which densification needs.
template <int PS, int LPP>
__global__ __launch_bounds__(256) void k_search(const SearchArgs a) {
    constexpr int NP = PS * PS;
    constexpr int GS = (NP + 15) / 16;
    constexpr int GPL = 16 / LPP;
    constexpr int PPL = GS * GPL;
    const int W = a.W, H = a.H;
    const int lane = threadIdx.x & (LPP - 1);
    const int N = a.nx * a.ny;
    int pi = (int)((blockIdx.x * 256u + threadIdx.x) / LPP);
    const bool valid = pi < N;
    if (!valid) pi = N - 1;    // idle groups shadow the last patch (no store): shuffles stay uniform

    const int ky = pi / a.nx, kx = pi - ky * a.nx;
    const int x0 = kx < a.nrx ? kx * a.st : W - PS;
    const int y0 = ky < a.nry ? ky * a.st : H - PS;

    double ui = 0.0, vi = 0.0;
    if (a.Un) {
        const double c = 0.5 * (PS - 1);
        double qx = (double)x0 + c, qy = (double)y0 + c;
        if (a.centre_map) { qx = (qx + 0.5) / 2.0 - 0.5; qy = (qy + 0.5) / 2.0 - 0.5; }
        else { qx = qx / 2.0; qy = qy / 2.0; }
        ui = 2.0 * bilin(a.Un, a.Wn, a.Hn, qx, qy);
        vi = 2.0 * bilin(a.Un + (size_t)a.Wn * a.Hn, a.Wn, a.Hn, qx, qy);
    }

    const double* __restrict__ J0 = a.J0;
    const double* __restrict__ J1 = a.J1;
    double T[PPL], gx[PPL], gy[PPL];
    int off[PPL];      // pixel offset py*W + px inside the frame
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int p = lane * PPL + k;
        if (p < NP) {
            const int py = p / PS, px = p - py * PS;
            const int x = x0 + px, y = y0 + py;
            const int xm = x > 0 ? x - 1 : 0, xp = x < W - 1 ? x + 1 : W - 1;
            const int ym = y > 0 ? y - 1 : 0, yp = y < H - 1 ? y + 1 : H - 1;
            T[k] = J0[y * W + x];
            const double dm = J0[ym * W + xp] - J0[ym * W + xm];
            const double d0 = J0[y * W + xp] - J0[y * W + xm];
            const double dp = J0[yp * W + xp] - J0[yp * W + xm];
            gx[k] = ((dm + 2.0 * d0) + dp) / 8.0;
            const double em = J0[yp * W + xm] - J0[ym * W + xm];
            const double e0 = J0[yp * W + x] - J0[ym * W + x];
            const double ep = J0[yp * W + xp] - J0[ym * W + xp];
            gy[k] = ((em + 2.0 * e0) + ep) / 8.0;
            off[k] = py * W + px;
        } else {
            T[k] = 0.0; gx[k] = 0.0; gy[k] = 0.0; off[k] = -1;
        }
    }
    const double h11 = csum_prod<GS, GPL, LPP>(gx, gx);
    const double h12 = csum_prod<GS, GPL, LPP>(gx, gy);
    const double h22 = csum_prod<GS, GPL, LPP>(gy, gy);
    const double sgx = csum<GS, GPL, LPP>(gx);
    const double sgy = csum<GS, GPL, LPP>(gy);
    const double a11 = h11 + a.lam, a22 = h22 + a.lam, a12 = h12;
    const double det = a11 * a22 - a12 * a12;
    const double inv_n = 1.0 / (double)NP;
    const double lim = (double)(W + H + 2 * PS + 4);

    double u = ui, v = vi, md = 0.0, moved = 0.0;
    for (int it = 0; it <= a.iters; ++it) {
        if (it == a.iters) {
            // reset test (Sec. 2.2 step 4), then one more warp at the final u
            const double eu = u - ui, ev = v - vi;
            moved = sqrt(eu * eu + ev * ev);
            if (moved > (double)PS) { u = ui; v = vi; }
        }
        const double fu = floor(u), fv = floor(v);
        const double ax = u - fu, ay = v - fv;
        const int iu = (int)fmin(fmax(fu, -lim), lim);
        const int iv = (int)fmin(fmax(fv, -lim), lim);
        double d[PPL];
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            if (off[k] >= 0) {
                const int py = (lane * PPL + k) / PS, px = (lane * PPL + k) - py * PS;
                const int xa = x0 + px + iu, ya = y0 + py + iv;
                const int c0 = clampi(xa, 0, W - 1), c1 = clampi(xa + 1, 0, W - 1);
                const int r0 = clampi(ya, 0, H - 1) * W, r1 = clampi(ya + 1, 0, H - 1) * W;
                const double top = (1.0 - ax) * J1[r0 + c0] + ax * J1[r0 + c1];
                const double bot = (1.0 - ax) * J1[r1 + c0] + ax * J1[r1 + c1];
                d[k] = ((1.0 - ay) * top + ay * bot) - T[k];
            } else {
                d[k] = 0.0;
            }
        }
        const double sd = csum<GS, GPL, LPP>(d);
        md = sd * inv_n;
        if (it == a.iters) break;
        // b = sum grad(T) (d - mean d): the mean-normalised residual (Sec. 2.1)
        const double b1 = csum_prod<GS, GPL, LPP>(gx, d) - md * sgx;
        const double b2 = csum_prod<GS, GPL, LPP>(gy, d) - md * sgy;
        u = u - (a22 * b1 - a12 * b2) / det;
        v = v - (a11 * b2 - a12 * b1) / det;
    }
    if (valid && lane == 0) {
        double* P = a.patch + (size_t)pi * 4;
        P[0] = u; P[1] = v; P[2] = md; P[3] = moved;
        a.uinit[(size_t)pi * 2] = ui;
        a.uinit[(size_t)pi * 2 + 1] = vi;
    }
}

// ------------------------------------------------------------ densification

__device__ __forceinline__ void cover_range(int x, int n, int ps, int st, int nr, int ntot,
                                            int& k0, int& k1, bool& flush) {
    const int lo = x - ps + 1;
    k0 = lo <= 0 ? 0 : (lo + st - 1) / st;
    k1 = x / st;
    if (k1 > nr - 1) k1 = nr - 1;
    flush = (ntot > nr) && (x >= n - ps);
}

// Eq. (3): per pixel, gather the covering patches in ascending patch index,
// weight each displacement by 1 / max(1, |d_i(x)|) with d_i the
// mean-normalised residual at that patch's displacement.
__global__ __launch_bounds__(256) void k_densify(const DensifyArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int W = a.W, H = a.H;
    if (x >= W || y >= H) return;
    int kx0, kx1, ky0, ky1;
    bool fx, fy;
    cover_range(x, W, a.ps, a.st, a.nrx, a.nx, kx0, kx1, fx);
    cover_range(y, H, a.ps, a.st, a.nry, a.ny, ky0, ky1, fy);
    const double j0 = a.J0[y * W + x];
    double su = 0.0, sv = 0.0, sw = 0.0;
    const int kyend = ky1 + (fy ? 1 : 0), kxend = kx1 + (fx ? 1 : 0);
    for (int jy = ky0; jy <= kyend; ++jy) {
        const int ky = jy <= ky1 ? jy : a.nry;
        for (int jx = kx0; jx <= kxend; ++jx) {
            const int kx = jx <= kx1 ? jx : a.nrx;
            const double* P = a.patch + (size_t)(ky * a.nx + kx) * 4;
            const double u = P[0], v = P[1];
            const double q = bilin(a.J1, W, H, (double)x + u, (double)y + v);
            const double d = a.raw_residual ? (q - j0) : ((q - j0) - P[2]);
            const double wgt = 1.0 / fmax(1.0, fabs(d));
            su = su + wgt * u;
            sv = sv + wgt * v;
            sw = sw + wgt;
        }
    }
    const double U = su / sw, V = sv / sw;
    const int g = y * W + x;
    a.U[g] = U;
    a.U[W * H + g] = V;
    if (a.J1w) a.J1w[g] = bilin(a.J1, W, H, (double)x + U, (double)y + V);
}

// -------------------------------------------------------- refinement setup

// Central differences [-1 0 1]/2 with replicated borders of the mean image
// (J0 + J1w)/2, of J1w - J0, and their second differences; the three data
// normalisations of Sec. 2.3.
__global__ __launch_bounds__(256) void k_prep(const PrepArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int W = a.W, H = a.H;
    if (x >= W || y >= H) return;
    const double* __restrict__ A = a.J0;
    const double* __restrict__ B = a.J1w;
    auto cx = [&](int v) { return clampi(v, 0, W - 1); };
    auto cy = [&](int v) { return clampi(v, 0, H - 1); };
    auto Ib = [&](int xx, int yy) { return 0.5 * (A[yy * W + xx] + B[yy * W + xx]); };
    auto Ixa = [&](int xx, int yy) { return (Ib(cx(xx + 1), yy) - Ib(cx(xx - 1), yy)) / 2.0; };
    auto Iya = [&](int xx, int yy) { return (Ib(xx, cy(yy + 1)) - Ib(xx, cy(yy - 1))) / 2.0; };
    const int xm = cx(x - 1), xp = cx(x + 1), ym = cy(y - 1), yp = cy(y + 1);
    const double Ix = Ixa(x, y);
    const double Iy = Iya(x, y);
    const int g = y * W + x;
    const double Iz = B[g] - A[g];
    const double Ixx = (Ixa(xp, y) - Ixa(xm, y)) / 2.0;
    const double Ixy = (Ixa(x, yp) - Ixa(x, ym)) / 2.0;
    const double Iyy = (Iya(x, yp) - Iya(x, ym)) / 2.0;
    const double Ixz = (B[y * W + xp] - B[y * W + xm]) / 2.0 - (A[y * W + xp] - A[y * W + xm]) / 2.0;
    const double Iyz = (B[yp * W + x] - B[ym * W + x]) / 2.0 - (A[yp * W + x] - A[ym * W + x]) / 2.0;
    const size_t n = (size_t)W * H;
    double* D = a.D;
    D[0 * n + g] = Ix;
    D[1 * n + g] = Iy;
    D[2 * n + g] = Iz;
    D[3 * n + g] = Ixx;
    D[4 * n + g] = Ixy;
    D[5 * n + g] = Iyy;
    D[6 * n + g] = Ixz;
    D[7 * n + g] = Iyz;
    D[8 * n + g] = 1.0 / ((Ix * Ix + Iy * Iy) + 0.01);
    D[9 * n + g] = 1.0 / ((Ixx * Ixx + Ixy * Ixy) + 0.01);
    D[10 * n + g] = 1.0 / ((Ixy * Ixy + Iyy * Iyy) + 0.01);
}

// --------------------------------------------------------------- refinement

// alpha / (2 sqrt(E_S + eps^2)) at (x, y) from forward differences of U + dU
// (zero across the last column / row).
__device__ __forceinline__ double smooth_weight(const RefineArgs& a, int x, int y) {
    const int W = a.W, H = a.H, g = y * W + x;
    const size_t n = (size_t)W * H;
    const double* U = a.U;
    const double* F = a.dUf;
    auto uu = [&](int i) { return F ? U[i] + F[i] : U[i]; };
    auto vv = [&](int i) { return F ? U[n + i] + F[n + i] : U[n + i]; };
    const double u0 = uu(g), v0 = vv(g);
    double dxu = 0.0, dyu = 0.0, dxv = 0.0, dyv = 0.0;
    if (x < W - 1) { dxu = uu(g + 1) - u0; dxv = vv(g + 1) - v0; }
    if (y < H - 1) { dyu = uu(g + W) - u0; dyv = vv(g + W) - v0; }
    const double es = ((dxu * dxu + dyu * dyu) + dxv * dxv) + dyv * dyv;
    return a.alpha / (2.0 * sqrt(es + a.eps * a.eps));
}

// One tile of the refinement.  The tile's core (TW x TH) is extended by
// nhalf pixels on every side that is not the image border; the sweeps run on
// the extended region in LDS, where an update can only be wrong at
// distance < j from a cut side after j half sweeps, so after nhalf half
// sweeps the core equals the untiled result exactly.  Each thread owns pairs
// of horizontally adjacent pixels (one of each colour), keeping their SOR
// coefficients in registers; LDS holds the increments and the edge weights.
template <int TW, int TH>
__global__ __launch_bounds__(256) void k_refine(const RefineArgs a) {
    constexpr int K = DIS_KMAX;
    constexpr int RWM = TW + 2 * K, RHM = TH + 2 * K;
    constexpr int LP = RWM + 1;                 // LDS row pitch
    constexpr int PWM = (RWM + 1) / 2;
    constexpr int PPT = (PWM * RHM + 255) / 256;
    __shared__ double s_du[RHM * LP], s_dv[RHM * LP], s_wr[RHM * LP], s_wd[RHM * LP];

    const int W = a.W, H = a.H;
    const size_t n = (size_t)W * H;
    const int kh = a.nhalf;
    const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
    const int cx0 = tx * TW, cy0 = ty * TH;
    const int cx1 = min(cx0 + TW, W), cy1 = min(cy0 + TH, H);
    const int rx0 = max(cx0 - kh, 0), ry0 = max(cy0 - kh, 0);
    const int rx1 = min(cx1 + kh, W), ry1 = min(cy1 + kh, H);
    const int RW = rx1 - rx0, RH = ry1 - ry0;

    for (int i = threadIdx.x; i < RW * RH; i += 256) {
        const int ly = i / RW, lx = i - ly * RW;
        const int x = rx0 + lx, y = ry0 + ly, g = y * W + x;
        const double ws = smooth_weight(a, x, y);
        const int l = ly * LP + lx;
        s_wr[l] = x < W - 1 ? ws : 0.0;
        s_wd[l] = y < H - 1 ? ws : 0.0;
        s_du[l] = a.dUin ? a.dUin[g] : 0.0;
        s_dv[l] = a.dUin ? a.dUin[n + g] : 0.0;
    }
    __syncthreads();

    const double om = a.omega, om1 = 1.0 - a.omega;
    const double eps2 = a.eps * a.eps;
    const int npw = (RW + 1) / 2;
    // per owned pixel: LDS index, neighbour mask, 4 edge weights, A12,
    // omega/(A11+S), omega/(A22+S), constant parts c1, c2
    int c_l[PPT][2], c_m[PPT][2];
    double c_wr[PPT][2], c_wl[PPT][2], c_wd[PPT][2], c_wu[PPT][2];
    double c_a12[PPT][2], c_i1[PPT][2], c_i2[PPT][2], c_c1[PPT][2], c_c2[PPT][2];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pr = threadIdx.x + k * 256;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            c_l[k][c] = -1;
            c_m[k][c] = 0;
            c_wr[k][c] = c_wl[k][c] = c_wd[k][c] = c_wu[k][c] = 0.0;
            c_a12[k][c] = c_i1[k][c] = c_i2[k][c] = c_c1[k][c] = c_c2[k][c] = 0.0;
            if (pr >= npw * RH) continue;
            const int ly = pr / npw, m = pr - ly * npw;
            const int y = ry0 + ly;
            const int lx = 2 * m + (((rx0 + y) & 1) ^ c);
            if (lx >= RW) continue;
            const int x = rx0 + lx, g = y * W + x;
            const int l = ly * LP + lx;
            const double* D = a.D;
            const double Ix = D[g], Iy = D[n + g], Iz = D[2 * n + g];
            const double Ixx = D[3 * n + g], Ixy = D[4 * n + g], Iyy = D[5 * n + g];
            const double Ixz = D[6 * n + g], Iyz = D[7 * n + g];
            const double b0 = D[8 * n + g], bx = D[9 * n + g], by = D[10 * n + g];
            const double fu = a.dUf ? a.dUf[g] : 0.0, fv = a.dUf ? a.dUf[n + g] : 0.0;
            const double ri = (Ix * fu + Iy * fv) + Iz;
            const double ei = b0 * (ri * ri);
            const double rx = (Ixx * fu + Ixy * fv) + Ixz;
            const double ry = (Ixy * fu + Iyy * fv) + Iyz;
            const double eg = bx * (rx * rx) + by * (ry * ry);
            const double pi_ = a.delta / (2.0 * sqrt(ei + eps2));
            const double pg = a.gamma / (2.0 * sqrt(eg + eps2));
            const double A11 = ((pi_ * b0) * Ix) * Ix + pg * (((bx * Ixx) * Ixx) + ((by * Ixy) * Ixy));
            const double A12 = ((pi_ * b0) * Ix) * Iy + pg * (((bx * Ixx) * Ixy) + ((by * Ixy) * Iyy));
            const double A22 = ((pi_ * b0) * Iy) * Iy + pg * (((bx * Ixy) * Ixy) + ((by * Iyy) * Iyy));
            const double B1 = ((pi_ * b0) * Ix) * Iz + pg * (((bx * Ixx) * Ixz) + ((by * Ixy) * Iyz));
            const double B2 = ((pi_ * b0) * Iy) * Iz + pg * (((bx * Ixy) * Ixz) + ((by * Iyy) * Iyz));
            // edges: right/down owned by this pixel, left/up by the neighbour;
            // neighbours outside the region (not the image) are dropped here,
            // which only disturbs pixels the erosion argument discards
            const bool hr = x < W - 1 && lx + 1 < RW, hl = x > 0 && lx > 0;
            const bool hd = y < H - 1 && ly + 1 < RH, hu = y > 0 && ly > 0;
            const double wr = hr ? s_wr[l] : 0.0, wl = hl ? s_wr[l - 1] : 0.0;
            const double wd = hd ? s_wd[l] : 0.0, wu = hu ? s_wd[l - LP] : 0.0;
            const double S = ((wr + wl) + wd) + wu;
            const double* U = a.U;
            const double Up = U[g], Vp = U[n + g];
            const double Ur = hr ? U[g + 1] : 0.0, Ul = hl ? U[g - 1] : 0.0;
            const double Ud = hd ? U[g + W] : 0.0, Uu = hu ? U[g - W] : 0.0;
            const double Vr = hr ? U[n + g + 1] : 0.0, Vl = hl ? U[n + g - 1] : 0.0;
            const double Vd = hd ? U[n + g + W] : 0.0, Vu = hu ? U[n + g - W] : 0.0;
            const double NU = ((wr * Ur + wl * Ul) + wd * Ud) + wu * Uu;
            const double NV = ((wr * Vr + wl * Vl) + wd * Vd) + wu * Vu;
            c_l[k][c] = l;
            c_m[k][c] = (hr ? 1 : 0) | (hl ? 2 : 0) | (hd ? 4 : 0) | (hu ? 8 : 0);
            c_wr[k][c] = wr; c_wl[k][c] = wl; c_wd[k][c] = wd; c_wu[k][c] = wu;
            c_a12[k][c] = A12;
            c_i1[k][c] = om / (A11 + S);
            c_i2[k][c] = om / (A22 + S);
            c_c1[k][c] = (NU - S * Up) - B1;
            c_c2[k][c] = (NV - S * Vp) - B2;
        }
    }

    // red-black half sweeps: colour 0 = (x + y) even, first
    for (int j = 0; j < kh; j += 2) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int l = c_l[k][c];
                if (l < 0) continue;
                const int m = c_m[k][c];
                const int lr = (m & 1) ? l + 1 : l, ll = (m & 2) ? l - 1 : l;
                const int ld = (m & 4) ? l + LP : l, lu = (m & 8) ? l - LP : l;
                const double du = s_du[l], dv = s_dv[l];
                const double nu = ((c_wr[k][c] * s_du[lr] + c_wl[k][c] * s_du[ll]) + c_wd[k][c] * s_du[ld]) +
                                  c_wu[k][c] * s_du[lu];
                const double dun = om1 * du + c_i1[k][c] * ((nu + c_c1[k][c]) - c_a12[k][c] * dv);
                const double nv = ((c_wr[k][c] * s_dv[lr] + c_wl[k][c] * s_dv[ll]) + c_wd[k][c] * s_dv[ld]) +
                                  c_wu[k][c] * s_dv[lu];
                const double dvn = om1 * dv + c_i2[k][c] * ((nv + c_c2[k][c]) - c_a12[k][c] * dun);
                s_du[l] = dun;
                s_dv[l] = dvn;
            }
            __syncthreads();
        }
    }

    const int CW = cx1 - cx0, CH = cy1 - cy0;
    for (int i = threadIdx.x; i < CW * CH; i += 256) {
        const int yy = i / CW, xx = i - yy * CW;
        const int x = cx0 + xx, y = cy0 + yy, g = y * W + x;
        const int l = (y - ry0) * LP + (x - rx0);
        const double du = s_du[l], dv = s_dv[l];
        a.dUout[g] = du;
        a.dUout[n + g] = dv;
        if (a.Uout) {
            a.Uout[g] = a.U[g] + du;
            a.Uout[n + g] = a.U[n + g] + dv;
        }
    }
}

// ----------------------------------------------------------------- upscale

__global__ __launch_bounds__(256) void k_upsample(const UpsArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.W || y >= a.H) return;
    double qx, qy;
    if (a.centre_map) { qx = ((double)x + 0.5) / a.f - 0.5; qy = ((double)y + 0.5) / a.f - 0.5; }
    else { qx = (double)x / a.f; qy = (double)y / a.f; }
    const double u = a.f * bilin(a.U, a.Ws, a.Hs, qx, qy);
    const double v = a.f * bilin(a.U + (size_t)a.Ws * a.Hs, a.Ws, a.Hs, qx, qy);
    const size_t g = (size_t)y * a.W + x, n = (size_t)a.W * a.H;
    if (a.out_f64) {
        ((double*)a.out)[g] = u;
        ((double*)a.out)[n + g] = v;
    } else {
        ((float*)a.out)[g] = (float)u;
        ((float*)a.out)[n + g] = (float)v;
    }
}

}  // namespace

// ------------------------------------------------------------ kernel table

const void* dis_kernel_pyramid() { return (const void*)&k_pyramid; }
const void* dis_kernel_densify() { return (const void*)&k_densify; }
const void* dis_kernel_prep() { return (const void*)&k_prep; }
const void* dis_kernel_upsample() { return (const void*)&k_upsample; }

#define DIS_SEARCH_CASE(PS_, LPP_) \
    if (ps == PS_ && lpp == LPP_) return (const void*)&k_search<PS_, LPP_>;

const void* dis_kernel_search(int ps, int lpp) {
    // instances whose per-lane pixel arrays fit the 256 architectural VGPRs
    DIS_SEARCH_CASE(4, 4) DIS_SEARCH_CASE(4, 8) DIS_SEARCH_CASE(4, 16)
    DIS_SEARCH_CASE(6, 4) DIS_SEARCH_CASE(6, 8) DIS_SEARCH_CASE(6, 16)
    DIS_SEARCH_CASE(8, 4) DIS_SEARCH_CASE(8, 8) DIS_SEARCH_CASE(8, 16)
    DIS_SEARCH_CASE(10, 8) DIS_SEARCH_CASE(10, 16)
    DIS_SEARCH_CASE(12, 8) DIS_SEARCH_CASE(12, 16)
    DIS_SEARCH_CASE(14, 16)
    DIS_SEARCH_CASE(16, 16)
    return nullptr;
}

int dis_refine_tile(int tile, int* tw, int* th) {
    switch (tile) {
        case 0: *tw = 32; *th = 16; return 1;
        case 1: *tw = 16; *th = 16; return 1;
        case 2: *tw = 64; *th = 8; return 1;
        default: return 0;
    }
}

const void* dis_kernel_refine(int tile) {
    switch (tile) {
        case 0: return (const void*)&k_refine<32, 16>;
        case 1: return (const void*)&k_refine<16, 16>;
        case 2: return (const void*)&k_refine<64, 8>;
        default: return nullptr;
    }
}
