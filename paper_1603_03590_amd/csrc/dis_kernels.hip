// HIP kernels of Dense Inverse Search optical flow for gfx950 (CDNA4).
//
// All arithmetic is float64: the pipeline (search, densification weights,
// robust refinement weights, upscaling) amplifies rounding noise by up to
// ~1e6, and on CDNA4 a float64 FMA issues at the same per-lane rate as an
// unpacked float32 one.  Frames arrive as float32 and are widened exactly.
//
// Built with -ffp-contract=off: every multiply-add the kernels fuse is an
// explicit fma(), so results do not depend on template instance or launch
// shape (the search's lanes-per-patch, the refinement's tile, the persistent
// or per-phase launch) -- all of them give the same bits.
//
// Each step is a device function over one block of work; the per-phase
// kernels and the persistent level kernel both call them.
#include <hip/hip_runtime.h>
#include "dis_internal.h"
#include "dis_lanes.h"
#include "dis_refine_tile.h"

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// Bilinear sample, pixel values at integer coordinates, taps clamped to the
// image.  Coordinates far outside are pulled to two pixels beyond the
// border first; that leaves the clamped taps (and so the value) unchanged.
template <class P>
__device__ __forceinline__ double bilin(P img, int W, int H, double x, double y) {
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

// One 256x32 tile of level a of frame f, channel c (512 threads): the tile's
// part of levels a+1..a+nlev.  Each thread owns a 4x4 block of level a (a
// wave covers 256 consecutive columns of four rows: every row of the tile is
// read as one 1 KB run) and forms its 2x2 of level a+1 and its pixel of level
// a+2 in registers; levels a+3.. come from LDS.  Every level pixel is the
// mean of a 2x2 block of the level below, summed row-major ((a+b)+c)+d, then
// scaled, whichever way it is reached.  Pixels outside level a read as 0;
// they never reach a stored pixel (levels are floor-halved).  The argument
// block is read once, before the tile's loads (in the table-driven launch it
// sits in memory).
__device__ __forceinline__ void pyramid_tile(const PyrArgs& A, int tile, int f, int c) {
    __shared__ double t2[8][65];
    __shared__ double t3[4][33];
    const int tiles_x = A.tiles_x, w0 = A.w0, h0 = A.h0, nlev = A.nlev, kind = A.src_kind, pitch = A.src_pitch;
    const double scale = A.scale;
    const size_t cs = (size_t)c * A.src_cstride;
    const void* src = f ? A.src[1] : A.src[0];
    double* lvl0 = f ? A.lvl0[1] : A.lvl0[0];
    double* dst[6];
    int ws[6], hs[6];
#pragma unroll
    for (int k = 1; k < 6; ++k) {
        dst[k] = f ? A.dst[1][k] : A.dst[0][k];
        ws[k] = A.ws[k];
        hs[k] = A.hs[k];
    }
    const int bx = tile % tiles_x, by = tile / tiles_x;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int x0 = bx * 256 + 4 * tx, y0 = by * 32 + 4 * ty;   // the thread's 4x4 block of level a
    // the loads are issued before any is used: one round of latency.  A row of
    // the block is one 16-byte load of a float32 frame (two of float64 data)
    // when the rows are 16-byte aligned and the block lies inside the level.
    const bool vec = ((reinterpret_cast<size_t>(src) | ((size_t)pitch * (kind == 1 ? 4 : 8)) |
                       (cs * (kind == 1 ? 4 : 8))) & 15) == 0;
    double v[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int y = y0 + r;
        const size_t g0 = cs + (size_t)y * pitch + x0;
        if (vec && y < h0 && x0 + 3 < w0) {
            if (kind == 1) {
                const float4 q4 = *reinterpret_cast<const float4*>((const float*)src + g0);
                v[r][0] = (double)q4.x; v[r][1] = (double)q4.y; v[r][2] = (double)q4.z; v[r][3] = (double)q4.w;
            } else {
                const double2 p0 = *reinterpret_cast<const double2*>((const double*)src + g0);
                const double2 p1 = *reinterpret_cast<const double2*>((const double*)src + g0 + 2);
                v[r][0] = p0.x; v[r][1] = p0.y; v[r][2] = p1.x; v[r][3] = p1.y;
            }
            continue;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int x = x0 + q;
            v[r][q] = 0.0;
            if (x < w0 && y < h0) {
                if (kind == 1)
                    v[r][q] = (double)((const float*)src)[g0 + q];
                else
                    v[r][q] = ((const double*)src)[g0 + q];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int x = x0 + q, y = y0 + r;
            v[r][q] = (x < w0 && y < h0) ? scale * v[r][q] : 0.0;
            if (lvl0 && x < w0 && y < h0) lvl0[((size_t)c * h0 + y) * w0 + x] = v[r][q];
        }
    }
    auto mean4 = [](double p, double q, double r, double s) { return 0.25 * (((p + q) + r) + s); };
    auto put = [&](int k, int xs, int ys, double val) {
        double* d = dst[k];
        if (d && xs < ws[k] && ys < hs[k]) d[((size_t)c * hs[k] + ys) * ws[k] + xs] = val;
    };
    // level a+1 (2x2) and a+2 (1) of the block
    double l1[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            l1[r][q] = mean4(v[2 * r][2 * q], v[2 * r][2 * q + 1], v[2 * r + 1][2 * q], v[2 * r + 1][2 * q + 1]);
            if (nlev >= 1) put(1, (x0 >> 1) + q, (y0 >> 1) + r, l1[r][q]);
        }
    const double l2 = mean4(l1[0][0], l1[0][1], l1[1][0], l1[1][1]);
    if (nlev >= 2) put(2, x0 >> 2, y0 >> 2, l2);
    if (nlev < 3) return;   // uniform over the block
    t2[ty][tx] = l2;
    __syncthreads();
    // level a+3: 32x4, level a+4: 16x2, level a+5: 8x1 of the tile
    if (threadIdx.x < 128) {
        const int ly = threadIdx.x >> 5, lx = threadIdx.x & 31;
        const double l3 = mean4(t2[2 * ly][2 * lx], t2[2 * ly][2 * lx + 1], t2[2 * ly + 1][2 * lx], t2[2 * ly + 1][2 * lx + 1]);
        put(3, bx * 32 + lx, by * 4 + ly, l3);
        t3[ly][lx] = l3;
    }
    if (nlev < 4) return;
    __syncthreads();
    double l4 = 0.0;
    if (threadIdx.x < 32) {
        const int ly = threadIdx.x >> 4, lx = threadIdx.x & 15;
        l4 = mean4(t3[2 * ly][2 * lx], t3[2 * ly][2 * lx + 1], t3[2 * ly + 1][2 * lx], t3[2 * ly + 1][2 * lx + 1]);
        put(4, bx * 16 + lx, by * 2 + ly, l4);
    }
    if (nlev < 5) return;
    // (t2 was last read before the barrier above)
    if (threadIdx.x < 32) t2[threadIdx.x >> 4][threadIdx.x & 15] = l4;
    __syncthreads();
    if (threadIdx.x < 8) {
        const int lx = threadIdx.x;
        put(5, bx * 8 + lx, by, mean4(t2[0][2 * lx], t2[0][2 * lx + 1], t2[1][2 * lx], t2[1][2 * lx + 1]));
    }
}

__global__ __launch_bounds__(512) void k_pyramid(const PyrArgs a) {
    if (blockIdx.x == 0 && blockIdx.y == 0)
        for (int i = threadIdx.x; i < a.nzero; i += 512) a.zero[i] = 0;
    pyramid_tile(a, blockIdx.x, blockIdx.y & 1, blockIdx.y >> 1);
}

// Pyramid passes of many pairs in one launch (tiles of pair j are
// start[j] .. start[j+1]-1).
__global__ __launch_bounds__(512) void k_pyramid_tab(const PyrTab T) {
    if (blockIdx.x == 0 && blockIdx.y == 0)
        for (int i = threadIdx.x; i < T.nzero; i += 512) T.zero[i] = 0;
    const int t = blockIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(T.blk[t]);
    pyramid_tile(T.tab[j], t - __builtin_amdgcn_readfirstlane(T.start[j]), blockIdx.y, 0);
}

// ------------------------------------------------------------------ search

// Canonical patch sums.  A patch's pixels p = 0..PS*PS-1 form NG groups of
// GS = ceil(PS*PS/NG) consecutive pixels (NG = 64 from 8x8 patches up, 16
// below; trailing groups may be empty); a group is summed sequentially (fma
// for products), then the NG group sums pairwise in a fixed binary tree.  A
// lane holds GPL = NG/LPP consecutive groups; the tree levels inside a lane are done in registers, the rest
// across the LPP lanes of the patch, pairing each block of lanes with the
// neighbouring block (every lane of a block holds the block's sum by then, so
// the pairing is the tree's): DPP moves within a row of 16 lanes, DPP row
// broadcasts across rows.  Every LPP therefore gives the same bits.
//
// tree_finish_n runs M such trees level by level (each value's tree is the
// one above, so every sum keeps its bits): the cross-lane latency of a level
// is paid once for all M sums instead of once per sum.
template <int GPL, int LPP, int M>
__device__ __forceinline__ void tree_finish_n(double (&g)[M][GPL], double (&s)[M]) {
#pragma unroll
    for (int step = 1; step < GPL; step <<= 1)
#pragma unroll
        for (int j = 0; j < GPL; j += 2 * step)
#pragma unroll
            for (int m = 0; m < M; ++m) g[m][j] = g[m][j] + g[m][j + step];
    double t[M];
#pragma unroll
    for (int m = 0; m < M; ++m) s[m] = g[m][0];
#define DIS_TREE_LEVEL(MOVE)                                          \
    _Pragma("unroll") for (int m = 0; m < M; ++m) t[m] = MOVE;        \
    _Pragma("unroll") for (int m = 0; m < M; ++m) s[m] = s[m] + t[m];
    if (LPP >= 2) { DIS_TREE_LEVEL(dpp_mov<0xB1>(s[m])) }    // quad_perm [1,0,3,2]
    if (LPP >= 4) { DIS_TREE_LEVEL(dpp_mov<0x4E>(s[m])) }    // quad_perm [2,3,0,1]
    if (LPP >= 8) { DIS_TREE_LEVEL(dpp_mov<0x141>(s[m])) }   // row_half_mirror
    if (LPP >= 16) { DIS_TREE_LEVEL(dpp_mov<0x140>(s[m])) }  // row_mirror
    // across rows: rows 1 and 3 add the last lane of rows 0 and 2 (by now
    // every lane of a row holds the row's sum), then row 3 adds lane 31; the
    // pairing is the tree's and a + b == b + a, so the bits are those of a
    // butterfly.  The other rows keep partial sums, and the patch's total,
    // in its last row, is read back to every lane.
    if (LPP >= 32) { DIS_TREE_LEVEL((dpp_bcast<0x142, 0xA>(s[m]))) }   // row_bcast:15 into rows 1, 3
    if (LPP >= 64) { DIS_TREE_LEVEL((dpp_bcast<0x143, 0x8>(s[m]))) }   // row_bcast:31 into row 3
#undef DIS_TREE_LEVEL
    if constexpr (LPP == 64) {
#pragma unroll
        for (int m = 0; m < M; ++m) s[m] = read_lane(s[m], 63);
    } else if constexpr (LPP == 32) {
        const bool upper = (threadIdx.x & 32) != 0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const double a = read_lane(s[m], 31), b = read_lane(s[m], 63);
            s[m] = upper ? b : a;
        }
    }
}

// Group sums of a lane: plain (v) or of products (a b, fma after the first).
template <int GS, int GPL>
__device__ __forceinline__ void group_sums(const double (&v)[GS * GPL], double (&g)[GPL]) {
#pragma unroll
    for (int j = 0; j < GPL; ++j) {
        double s = v[j * GS];
#pragma unroll
        for (int k = 1; k < GS; ++k) s = s + v[j * GS + k];
        g[j] = s;
    }
}

template <int GS, int GPL>
__device__ __forceinline__ void group_sums(const double (&a)[GS * GPL], const double (&b)[GS * GPL],
                                           double (&g)[GPL]) {
#pragma unroll
    for (int j = 0; j < GPL; ++j) {
        double s = a[j * GS] * b[j * GS];
#pragma unroll
        for (int k = 1; k < GS; ++k) s = fma(a[j * GS + k], b[j * GS + k], s);
        g[j] = s;
    }
}

template <int GS, int GPL, int LPP>
__device__ __forceinline__ double csum(const double (&v)[GS * GPL]) {
    double g[1][GPL], s[1];
    group_sums<GS, GPL>(v, g[0]);
    tree_finish_n<GPL, LPP, 1>(g, s);
    return s[0];
}

constexpr int isqrt_floor(int v, int r = 0) { return (r + 1) * (r + 1) > v ? r : isqrt_floor(v, r + 1); }

// LDS copy of the second frame around each patch's initial position: a
// square of PS + 1 + 2R pixels per channel (indices clamped to the image as
// the bilinear taps clamp them), R as large as 48 KB per block allows (at
// most 6).  While the patch's integer displacement stays within R of its
// start the warps read LDS; beyond, global memory.  Same values either way.
template <int PS, int LPP, int NC = 1>
struct SearchWin {
    static constexpr int GROUPS = 256 / LPP;
    static constexpr int FIT = (isqrt_floor(48 * 1024 / 8 / GROUPS / NC) - PS - 1) / 2;
    static constexpr int R = LPP < 8 ? 0 : (FIT < 0 ? 0 : (FIT > 6 ? 6 : FIT));
    static constexpr int WS = PS + 1 + 2 * R;
};

// One block of 256 threads = 256/LPP patches, LPP lanes per patch.  Patch
// corners, initialisation (Sec. 2.2 steps 1-2), template and Sobel/8
// gradients, the precomputed 2x2 Hessian, theta_it inverse-compositional
// updates u <- u - H^-1 sum grad(T) r (Suppl. A), the reset test of step 4,
// and the mean residual at the final u, which densification needs.  With NC
// colour channels (App. B i) the Hessian and the right-hand side are sums of
// the per-channel ones (channel 0 first), each channel mean-normalised on
// its own.
template <int PS, int LPP, int NC = 1>
__device__ __forceinline__ void search_block(const SearchArgs& a, int block) {
    constexpr int NP = PS * PS;
    constexpr int NG = NP >= 64 ? 64 : 16;
    static_assert(LPP <= NG, "more lanes than groups");
    constexpr int GS = (NP + NG - 1) / NG;
    constexpr int GPL = NG / LPP;
    constexpr int PPL = GS * GPL;
    const int W = a.W, H = a.H;
    const size_t n = (size_t)W * H;
    const int lane = threadIdx.x & (LPP - 1);
    const int N = a.nx * a.ny;
    int pi = (int)((block * 256u + threadIdx.x) / LPP);
    const bool valid = pi < N;
    if (!valid) pi = N - 1;    // idle groups shadow the last patch (no store): DPP stays uniform

    const int ky = pi / a.nx, kx = pi - ky * a.nx;
    const int x0 = kx < a.nrx ? kx * a.st : W - PS;
    const int y0 = ky < a.nry ? ky * a.st : H - PS;

    // taps of the coarser flow at the patch centre, requested before the
    // template so that both rounds of loads are in flight together (the
    // value is bilin() of the coarser flow, combined below in the same order)
    const bool has_un = a.Un != nullptr;
    double u00, u01, u10, u11, v00, v01, v10, v11, bax, bay;
    {
        const auto* Up = dis_global(has_un ? a.Un : a.J0);
        const int Wn = has_un ? a.Wn : W, Hn = has_un ? a.Hn : H;
        const double c = 0.5 * (PS - 1);
        double qx = (double)x0 + c, qy = (double)y0 + c;
        if (a.centre_map) { qx = (qx + 0.5) / 2.0 - 0.5; qy = (qy + 0.5) / 2.0 - 0.5; }
        else { qx = qx / 2.0; qy = qy / 2.0; }
        double xf = floor(qx), yf = floor(qy);
        bax = qx - xf;
        bay = qy - yf;
        xf = fmin(fmax(xf, -2.0), (double)Wn + 1.0);
        yf = fmin(fmax(yf, -2.0), (double)Hn + 1.0);
        const int xi = (int)xf, yi = (int)yf;
        const int c0 = clampi(xi, 0, Wn - 1), c1 = clampi(xi + 1, 0, Wn - 1);
        const int r0 = clampi(yi, 0, Hn - 1) * Wn, r1 = clampi(yi + 1, 0, Hn - 1) * Wn;
        const auto* Vp = Up + (has_un ? (size_t)Wn * Hn : 0);
        u00 = Up[r0 + c0]; u01 = Up[r0 + c1]; u10 = Up[r1 + c0]; u11 = Up[r1 + c1];
        v00 = Vp[r0 + c0]; v01 = Vp[r0 + c1]; v10 = Vp[r1 + c0]; v11 = Vp[r1 + c1];
    }

    double T[NC][PPL], gx[NC][PPL], gy[NC][PPL];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) {
        const auto* __restrict__ J0 = dis_global(a.J0) + ch * n;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int p = lane * PPL + k;
            if (p < NP) {
                const int py = p / PS, px = p - py * PS;
                const int x = x0 + px, y = y0 + py;
                const int xm = x > 0 ? x - 1 : 0, xp = x < W - 1 ? x + 1 : W - 1;
                const int ym = y > 0 ? y - 1 : 0, yp = y < H - 1 ? y + 1 : H - 1;
                T[ch][k] = J0[y * W + x];
                const double dm = J0[ym * W + xp] - J0[ym * W + xm];
                const double d0 = J0[y * W + xp] - J0[y * W + xm];
                const double dp = J0[yp * W + xp] - J0[yp * W + xm];
                gx[ch][k] = ((dm + 2.0 * d0) + dp) / 8.0;
                const double em = J0[yp * W + xm] - J0[ym * W + xm];
                const double e0 = J0[yp * W + x] - J0[ym * W + x];
                const double ep = J0[yp * W + xp] - J0[ym * W + xp];
                gy[ch][k] = ((em + 2.0 * e0) + ep) / 8.0;
            } else {
                T[ch][k] = 0.0; gx[ch][k] = 0.0; gy[ch][k] = 0.0;
            }
        }
    }
    // H' (channel sums, channel 0 first) and the gradient sums, all of one
    // channel's five trees at once
    double h11 = 0.0, h12 = 0.0, h22 = 0.0, sgx[NC], sgy[NC];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) {
        double g5[5][GPL], s5[5];
        group_sums<GS, GPL>(gx[ch], gx[ch], g5[0]);
        group_sums<GS, GPL>(gx[ch], gy[ch], g5[1]);
        group_sums<GS, GPL>(gy[ch], gy[ch], g5[2]);
        group_sums<GS, GPL>(gx[ch], g5[3]);
        group_sums<GS, GPL>(gy[ch], g5[4]);
        tree_finish_n<GPL, LPP, 5>(g5, s5);
        if (ch == 0) { h11 = s5[0]; h12 = s5[1]; h22 = s5[2]; }
        else { h11 = h11 + s5[0]; h12 = h12 + s5[1]; h22 = h22 + s5[2]; }
        sgx[ch] = s5[3];
        sgy[ch] = s5[4];
    }
    double ui = 0.0, vi = 0.0;
    if (has_un) {
        ui = 2.0 * ((1.0 - bay) * ((1.0 - bax) * u00 + bax * u01) + bay * ((1.0 - bax) * u10 + bax * u11));
        vi = 2.0 * ((1.0 - bay) * ((1.0 - bax) * v00 + bax * v01) + bay * ((1.0 - bax) * v10 + bax * v11));
    }
    const double a11 = h11 + a.lam, a22 = h22 + a.lam, a12 = h12;
    const double idet = 1.0 / (a11 * a22 - a12 * a12);
    // H^-1 b = (m11 b1 + m12 b2, m12 b1 + m22 b2)
    const double m11 = a22 * idet, m12 = -a12 * idet, m22 = a11 * idet;
    const double inv_n = 1.0 / (double)NP;
    const double lim = (double)(W + H + 2 * PS + 4);

    // the window of this patch (see SearchWin), one per channel
    using SW = SearchWin<PS, LPP, NC>;
    constexpr int R = SW::R, WS = SW::WS;
    __shared__ double s_win[R > 0 ? NC * SW::GROUPS * WS * WS : 1];
    const int iu0 = (int)fmin(fmax(floor(ui), -lim), lim), iv0 = (int)fmin(fmax(floor(vi), -lim), lim);
    double* win = s_win + (size_t)(threadIdx.x / LPP) * NC * WS * WS;
    if constexpr (R > 0) {
        const int wx = x0 + iu0 - R, wy = y0 + iv0 - R;
        // every load of a lane is issued before the first store, so the
        // window costs one round of memory latency, not one per element
        constexpr int NW = (WS * WS + LPP - 1) / LPP;
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) {
            double wv[NW];
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                const int i = lane + k * LPP;
                const int Y = i / WS, X = i - Y * WS;
                wv[k] = i < WS * WS ? dis_global(a.J1)[ch * n + clampi(wy + Y, 0, H - 1) * W + clampi(wx + X, 0, W - 1)] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                const int i = lane + k * LPP;
                if (i < WS * WS) win[ch * WS * WS + i] = wv[k];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }

    double u = ui, v = vi, md0 = 0.0, moved = 0.0;
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
        const bool in_win = R > 0 && iu - iu0 >= -R && iu - iu0 <= R && iv - iv0 >= -R && iv - iv0 <= R;
        double b1 = 0.0, b2 = 0.0;
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) {
            double d[PPL];
            if (in_win) {
                const double* wc = win + ch * WS * WS;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    const int p = lane * PPL + k;
                    if (p < NP) {
                        const int py = p / PS, px = p - py * PS;
                        const double* c = wc + (py + iv - iv0 + R) * WS + (px + iu - iu0 + R);
                        const double top = (1.0 - ax) * c[0] + ax * c[1];
                        const double bot = (1.0 - ax) * c[WS] + ax * c[WS + 1];
                        d[k] = ((1.0 - ay) * top + ay * bot) - T[ch][k];
                    } else {
                        d[k] = 0.0;
                    }
                }
            } else {
                const auto* __restrict__ J1 = dis_global(a.J1) + ch * n;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    const int p = lane * PPL + k;
                    if (p < NP) {
                        const int py = p / PS, px = p - py * PS;
                        const int xa = x0 + px + iu, ya = y0 + py + iv;
                        const int c0 = clampi(xa, 0, W - 1), c1 = clampi(xa + 1, 0, W - 1);
                        const int r0 = clampi(ya, 0, H - 1) * W, r1 = clampi(ya + 1, 0, H - 1) * W;
                        const double top = (1.0 - ax) * J1[r0 + c0] + ax * J1[r0 + c1];
                        const double bot = (1.0 - ax) * J1[r1 + c0] + ax * J1[r1 + c1];
                        d[k] = ((1.0 - ay) * top + ay * bot) - T[ch][k];
                    } else {
                        d[k] = 0.0;
                    }
                }
            }
            double c1, c2;
            if (a.norm == 0 && it < a.iters) {
                // b = sum grad(T) (d - mean d): the mean-normalised residual
                // (Sec. 2.1); the three sums share one tree pass
                double g3[3][GPL], s3[3];
                group_sums<GS, GPL>(d, g3[0]);
                group_sums<GS, GPL>(gx[ch], d, g3[1]);
                group_sums<GS, GPL>(gy[ch], d, g3[2]);
                tree_finish_n<GPL, LPP, 3>(g3, s3);
                const double md = s3[0] * inv_n;
                c1 = s3[1] - md * sgx[ch];
                c2 = s3[2] - md * sgy[ch];
            } else {
                // the final warp (only the mean residual), or a robust norm
                const double sd = csum<GS, GPL, LPP>(d);
                const double md = sd * inv_n;
                if (it == a.iters) {
                    if (ch == 0) md0 = md;
                    if (NC > 1 && valid && lane == 0) dis_global(a.mdc)[(size_t)pi * NC + ch] = md;
                    continue;
                }
                // App. B iii: each mean-normalised residual e is transformed so
                // that its square is the L1 or the Huber penalty of e
                double r[PPL];
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    const int p = lane * PPL + k;
                    const double e = d[k] - md;
                    const double ae = fabs(e);
                    double t;
                    if (a.norm == 1) t = sqrt(ae);
                    else t = ae < a.huber_b ? ae : sqrt(2.0 * a.huber_b * ae - a.huber_b * a.huber_b);
                    r[k] = p < NP ? copysign(t, e) : 0.0;
                }
                double g2[2][GPL], s2[2];
                group_sums<GS, GPL>(gx[ch], r, g2[0]);
                group_sums<GS, GPL>(gy[ch], r, g2[1]);
                tree_finish_n<GPL, LPP, 2>(g2, s2);
                c1 = s2[0];
                c2 = s2[1];
            }
            if (ch == 0) { b1 = c1; b2 = c2; }
            else { b1 = b1 + c1; b2 = b2 + c2; }
        }
        if (it == a.iters) break;
        if (a.stereo) {
            u = u - b1 / a11;   // App. I: one degree of freedom, v stays at its start (zero)
        } else {
            u = u - (m11 * b1 + m12 * b2);
            v = v - (m12 * b1 + m22 * b2);
        }
    }
    if (valid && lane == 0) {
        auto* P = dis_global(a.patch) + (size_t)pi * 4;
        P[0] = u; P[1] = v; P[2] = md0; P[3] = moved;
        dis_global(a.uinit)[(size_t)pi * 2] = ui;
        dis_global(a.uinit)[(size_t)pi * 2 + 1] = vi;
    }
}

#include "dis_search_rows.h"

// ------------------------------------------------------------ densification

__device__ __forceinline__ void cover_range(int x, int n, int ps, int st, int nr, int ntot,
                                            int& k0, int& k1, bool& flush) {
    const int lo = x - ps + 1;
    k0 = lo <= 0 ? 0 : (lo + st - 1) / st;
    k1 = x / st;
    if (k1 > nr - 1) k1 = nr - 1;
    flush = (ntot > nr) && (x >= n - ps);
}

// Eq. (3) at pixel (x, y): the covering patches in ascending patch index,
// each displacement weighted by 1 / max(1, |d_i(x)|) with d_i the
// mean-normalised residual at that patch's displacement (with colour
// frames, App. B i: the Euclidean norm over the channels of the per-channel
// residuals).  Returns the displacement average U, V and the weight sum.
template <bool COLOUR = false>
__device__ __forceinline__ void densify_pixel(const DensifyArgs& a, int x, int y, double& U, double& V,
                                              double& sw) {
    const int W = a.W, H = a.H;
    const size_t n = (size_t)W * H;
    int kx0, kx1, ky0, ky1;
    bool fx, fy;
    cover_range(x, W, a.ps, a.st, a.nrx, a.nx, kx0, kx1, fx);
    cover_range(y, H, a.ps, a.st, a.nry, a.ny, ky0, ky1, fy);
    const double j0 = dis_global(a.J0)[y * W + x];
    double su = 0.0, sv = 0.0;
    sw = 0.0;
    const int kyend = ky1 + (fy ? 1 : 0), kxend = kx1 + (fx ? 1 : 0);
    for (int jy = ky0; jy <= kyend; ++jy) {
        const int ky = jy <= ky1 ? jy : a.nry;
        for (int jx = kx0; jx <= kxend; ++jx) {
            const int kx = jx <= kx1 ? jx : a.nrx;
            const int i = ky * a.nx + kx;
            const auto* P = dis_global(a.patch) + (size_t)i * 4;
            const double u = P[0], v = P[1];
            const double q = bilin(dis_global(a.J1), W, H, (double)x + u, (double)y + v);
            double ad;
            if constexpr (!COLOUR) {
                ad = fabs(a.raw_residual ? (q - j0) : ((q - j0) - P[2]));
            } else {
                double ss = 0.0;
                for (int ch = 0; ch < a.nc; ++ch) {
                    const double qc = ch ? bilin(dis_global(a.J1) + ch * n, W, H, (double)x + u, (double)y + v) : q;
                    const double jc = dis_global(a.J0)[ch * n + (size_t)y * W + x];
                    const double dc = a.raw_residual ? (qc - jc) : ((qc - jc) - dis_global(a.mdc)[(size_t)i * a.nc + ch]);
                    ss = ch ? ss + dc * dc : dc * dc;
                }
                ad = sqrt(ss);
            }
            const double wgt = 1.0 / fmax(1.0, ad);
            su = su + wgt * u;
            sv = sv + wgt * v;
            sw = sw + wgt;
        }
    }
    U = su / sw;
    V = sv / sw;
}

// Eq. (3) on a 64x4 block, then the second frame (every channel) warped by
// the dense flow, for the refinement.
template <bool COLOUR = false>
__device__ __forceinline__ void densify_block(const DensifyArgs& a, int bx, int by) {
    const int x = bx * 64 + (threadIdx.x & 63);
    const int y = by * 4 + (threadIdx.x >> 6);
    const int W = a.W, H = a.H;
    if (x >= W || y >= H) return;
    double U, V, sw;
    densify_pixel<COLOUR>(a, x, y, U, V, sw);
    const int g = y * W + x;
    if (a.Z) dis_global(a.Z)[g] = sw;
    dis_global(a.U)[g] = U;
    dis_global(a.U)[W * H + g] = V;
    if (a.J1w) {
        if constexpr (!COLOUR) {
            dis_global(a.J1w)[g] = bilin(dis_global(a.J1), W, H, (double)x + U, (double)y + V);
        } else {
            for (int ch = 0; ch < a.nc; ++ch)
                dis_global(a.J1w)[(size_t)ch * W * H + g] = bilin(dis_global(a.J1) + (size_t)ch * W * H, W, H, (double)x + U, (double)y + V);
        }
    }
}

// Linearisation of the refinement (Sec. 2.3) for colour frames: per pixel
// and channel the central differences of (J0 + J1w)/2 and of J1w - J0 with
// replicated borders, and the three normalisers, as [nc][11][H][W].  The
// refinement tile then sums the data terms over the channels.
__global__ __launch_bounds__(256) void k_colour_lin(const LevelLaunch L) {
    const RefineArgs& a = L.pairs[0].ra;
    const int W = a.W, H = a.H;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const size_t n = (size_t)W * H;
    const int xm = max(x - 1, 0), xp = min(x + 1, W - 1);
    const int ym = max(y - 1, 0), yp = min(y + 1, H - 1);
    for (int ch = 0; ch < a.nc; ++ch) {
        const auto* t0 = dis_global(a.J0) + ch * n;
        const auto* t1 = dis_global(a.J1w) + ch * n;
        auto Ib = [&](int xx, int yy) { const size_t l = (size_t)yy * W + xx; return 0.5 * (t0[l] + t1[l]); };
        auto Ixa = [&](int xx, int yy) { return (Ib(min(xx + 1, W - 1), yy) - Ib(max(xx - 1, 0), yy)) / 2.0; };
        auto Iya = [&](int xx, int yy) { return (Ib(xx, min(yy + 1, H - 1)) - Ib(xx, max(yy - 1, 0))) / 2.0; };
        const size_t gi = (size_t)y * W + x;
        const double Ix = Ixa(x, y), Iy = Iya(x, y);
        const double Iz = t1[gi] - t0[gi];
        const double Ixx = (Ixa(xp, y) - Ixa(xm, y)) / 2.0;
        const double Ixy = (Ixa(x, yp) - Ixa(x, ym)) / 2.0;
        const double Iyy = (Iya(x, yp) - Iya(x, ym)) / 2.0;
        const size_t lxp = (size_t)y * W + xp, lxm = (size_t)y * W + xm;
        const size_t lyp = (size_t)yp * W + x, lym = (size_t)ym * W + x;
        const double Ixz = (t1[lxp] - t1[lxm]) / 2.0 - (t0[lxp] - t0[lxm]) / 2.0;
        const double Iyz = (t1[lyp] - t1[lym]) / 2.0 - (t0[lyp] - t0[lym]) / 2.0;
        auto* Lo = dis_global(a.lin) + (size_t)ch * 11 * n + gi;
        Lo[0] = Ix; Lo[n] = Iy; Lo[2 * n] = Iz; Lo[3 * n] = Ixx; Lo[4 * n] = Ixy; Lo[5 * n] = Iyy;
        Lo[6 * n] = Ixz; Lo[7 * n] = Iyz;
        Lo[8 * n] = 1.0 / ((Ix * Ix + Iy * Iy) + 0.01);
        Lo[9 * n] = 1.0 / ((Ixx * Ixx + Ixy * Ixy) + 0.01);
        Lo[10 * n] = 1.0 / ((Ixy * Ixy + Iyy * Iyy) + 0.01);
    }
}

// ------------------------------------------- forward-backward densification

// Displaced-corner cell of patch j of a direction, or -1 when its displaced
// square cannot reach the level (floor division by the patch size).
__device__ __forceinline__ int fb_cell(const DensifyArgs& o, int j, int Wc, int Hc) {
    const int ky = j / o.nx, kx = j - ky * o.nx;
    const int x0 = kx < o.nrx ? kx * o.st : o.W - o.ps;
    const int y0 = ky < o.nry ? ky * o.st : o.H - o.ps;
    const double* P = o.patch + (size_t)j * 4;
    const double fx = floor((double)x0 + P[0]), fy = floor((double)y0 + P[1]);
    const double cxd = floor(fx / o.ps) + 1.0, cyd = floor(fy / o.ps) + 1.0;
    if (!(cxd >= 0.0 && cxd < (double)Wc && cyd >= 0.0 && cyd < (double)Hc)) return -1;
    return (int)cyd * Wc + (int)cxd;
}

__global__ __launch_bounds__(256) void k_fb_count(const FbLaunch F) {
    const int d = blockIdx.y;
    const DensifyArgs& o = F.L.pairs[1 - d].da;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= o.nx * o.ny) return;
    const int c = fb_cell(o, j, F.Wc, F.Hc);
    if (c >= 0) atomicAdd(F.bins[d].count + c, 1);
}

// exclusive prefix sum of the counts (one block per direction); clears the
// counts for the next use
__global__ __launch_bounds__(1024) void k_fb_scan(const FbLaunch F) {
    __shared__ int part[1024];
    const FbBins& B = F.bins[blockIdx.y];
    const int n = F.Wc * F.Hc;
    const int per = (n + 1023) / 1024;
    const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
    int sum = 0;
    for (int i = lo; i < hi; ++i) sum += B.count[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int i = lo; i < hi; ++i) {
        const int c = B.count[i];
        B.start[i] = run;
        B.cursor[i] = run;
        B.count[i] = 0;
        run += c;
    }
    if (threadIdx.x == 1023) B.start[n] = part[1023];
}

__global__ __launch_bounds__(256) void k_fb_scatter(const FbLaunch F) {
    const int d = blockIdx.y;
    const DensifyArgs& o = F.L.pairs[1 - d].da;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= o.nx * o.ny) return;
    const int c = fb_cell(o, j, F.Wc, F.Hc);
    if (c >= 0) F.bins[d].list[atomicAdd(F.bins[d].cursor + c, 1)] = j;
}

// Eq. (3) merged over both directions (App. B ii) for the flow of direction
// d: its own covering patches in ascending index, then the other
// direction's patches whose displaced square covers the pixel, in ascending
// index (sorted here, the bins hold them in arrival order), each voting -u
// with the residual of its template sampled bilinearly at x - u.
__global__ __launch_bounds__(256) void k_fb_densify(const FbLaunch F) {
    const int d = blockIdx.z;
    const DensifyArgs& a = F.L.pairs[d].da;
    const DensifyArgs& o = F.L.pairs[1 - d].da;
    const FbBins& B = F.bins[d];
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int W = a.W, H = a.H;
    if (x >= W || y >= H) return;
    double su = 0.0, sv = 0.0, sw = 0.0;
    {
        // own patches, as Eq. (3) (the sums, not yet divided)
        int kx0, kx1, ky0, ky1;
        bool fx, fy;
        cover_range(x, W, a.ps, a.st, a.nrx, a.nx, kx0, kx1, fx);
        cover_range(y, H, a.ps, a.st, a.nry, a.ny, ky0, ky1, fy);
        const double j0 = dis_global(a.J0)[y * W + x];
        const int kyend = ky1 + (fy ? 1 : 0), kxend = kx1 + (fx ? 1 : 0);
        for (int jy = ky0; jy <= kyend; ++jy) {
            const int ky = jy <= ky1 ? jy : a.nry;
            for (int jx = kx0; jx <= kxend; ++jx) {
                const int kx = jx <= kx1 ? jx : a.nrx;
                const auto* P = dis_global(a.patch) + (size_t)(ky * a.nx + kx) * 4;
                const double u = P[0], v = P[1];
                const double q = bilin(dis_global(a.J1), W, H, (double)x + u, (double)y + v);
                const double dd = a.raw_residual ? (q - j0) : ((q - j0) - P[2]);
                const double wgt = 1.0 / fmax(1.0, fabs(dd));
                su = su + wgt * u;
                sv = sv + wgt * v;
                sw = sw + wgt;
            }
        }
    }
    // candidates of the other direction: 2 x 2 cells
    const int ps = o.ps;
    const double xr = (double)x, yr = (double)y;
    const double j0 = dis_global(a.J0)[y * W + x];
    auto covers = [&](int j, double& uj, double& vj, double& md) {
        const int ky = j / o.nx, kx = j - ky * o.nx;
        const int x0 = kx < o.nrx ? kx * o.st : o.W - ps;
        const int y0 = ky < o.nry ? ky * o.st : o.H - ps;
        const auto* P = dis_global(o.patch) + (size_t)j * 4;
        uj = P[0]; vj = P[1]; md = P[2];
        const double xa = (double)x0 + uj, ya = (double)y0 + vj;
        return xa <= xr && xr <= (double)x0 + (double)(ps - 1) + uj && ya <= yr &&
               yr <= (double)y0 + (double)(ps - 1) + vj;
    };
    const int cx1 = x / ps + 1, cy1 = y / ps + 1;
    int cand[DIS_FB_MAXCAND];
    int nc = 0;
    bool overflow = false;
    for (int cy = cy1 - 1; cy <= cy1; ++cy)
        for (int cx = cx1 - 1; cx <= cx1; ++cx) {
            const int c = cy * F.Wc + cx;
            for (int t = dis_global(B.start)[c]; t < dis_global(B.start)[c + 1]; ++t) {
                const int j = dis_global(B.list)[t];
                double uj, vj, md;
                if (!covers(j, uj, vj, md)) continue;
                if (nc == DIS_FB_MAXCAND) { overflow = true; continue; }
                // insertion into the ascending list
                int q = nc++;
                while (q > 0 && cand[q - 1] > j) { cand[q] = cand[q - 1]; --q; }
                cand[q] = j;
            }
        }
    auto vote = [&](int j) {
        double uj, vj, md;
        covers(j, uj, vj, md);
        const double tv = bilin(dis_global(o.J0), W, H, xr - uj, yr - vj);   // the other direction's template frame
        const double dd = a.raw_residual ? (j0 - tv) : ((j0 - tv) - md);
        const double wgt = 1.0 / fmax(1.0, fabs(dd));
        su = su - wgt * uj;
        sv = sv - wgt * vj;
        sw = sw + wgt;
    };
    if (!overflow) {
        for (int q = 0; q < nc; ++q) vote(cand[q]);
    } else {
        // more covering patches than the sorted list holds: ascending order by
        // repeated selection over the cells
        int prev = -1;
        for (;;) {
            int best = 0x7fffffff;
            for (int cy = cy1 - 1; cy <= cy1; ++cy)
                for (int cx = cx1 - 1; cx <= cx1; ++cx) {
                    const int c = cy * F.Wc + cx;
                    for (int t = dis_global(B.start)[c]; t < dis_global(B.start)[c + 1]; ++t) {
                        const int j = dis_global(B.list)[t];
                        double uj, vj, md;
                        if (j > prev && j < best && covers(j, uj, vj, md)) best = j;
                    }
                }
            if (best == 0x7fffffff) break;
            vote(best);
            prev = best;
        }
    }
    const double Uo = su / sw, Vo = sv / sw;
    const int g = y * W + x;
    dis_global(a.U)[g] = Uo;
    dis_global(a.U)[W * H + g] = Vo;
    if (a.J1w) dis_global(a.J1w)[g] = bilin(dis_global(a.J1), W, H, xr + Uo, yr + Vo);
}

// --------------------------------------------------------------- refinement

using dis_tile::RefineSmem;

// One tile of one fixed-point step of the refinement (Sec. 2.3).  The core
// is extended by nhalf pixels on every side that is not the image border;
// the sweeps run on that region in LDS, where an update can be wrong only at
// distance < j from a cut side after j half sweeps, so after nhalf half
// sweeps the core equals the untiled result exactly.  Each of the NT threads
// owns pairs of horizontally adjacent pixels (one of each colour) and keeps
// their SOR coefficients in registers; LDS holds the increments, the edge
// weights and U.  Every global read is issued in one round at the start.
template <int TW, int TH, int NT, bool COLOUR = false, bool LEAN = false>
__device__ __forceinline__ void refine_tile(const RefineArgs& a, int tile, RefineSmem<TW, TH, DIS_KMAX, LEAN>& sm) {
    using S = RefineSmem<TW, TH, DIS_KMAX, LEAN>;
    using Shape = dis_tile::TileShape<TW, TH, NT, DIS_KMAX, LEAN>;
    constexpr int LP = S::LP;
    constexpr int PPT = Shape::PPT;
    constexpr bool kStage = Shape::kStage;
    const int kh = __builtin_amdgcn_readfirstlane(a.nhalf);   // steers a loop with barriers
    const dis_tile::TileGeom g = dis_tile::tile_geom<TW, TH>(a.W, a.H, a.tiles_x, tile, kh);
    const int W = g.W, H = g.H;
    const size_t n = (size_t)W * H;
    const int rx0 = g.rx0, ry0 = g.ry0, RW = g.RW, RH = g.RH;
    const int cx0 = g.cx0, cy0 = g.cy0, cx1 = g.cx1, cy1 = g.cy1;
    const auto* __restrict__ Din = dis_global(a.dUin);
    const double om1 = 1.0 - a.omega;
    const bool stereo = a.stereo != 0;

    dis_tile::TileCoef<PPT> C;
    double s_iu[Shape::NS][2], s_iv[Shape::NS][2];
    // the sweeps below update only pixels closer to the core than the number
    // of half sweeps they run
    dis_tile::refine_setup<TW, TH, NT, DIS_KMAX, COLOUR, LEAN>(a, g, sm, C, s_iu, s_iv, 2 * ((kh + 1) / 2) - 1);
    __syncthreads();   // the image tile is dead from here on
    // 4. sweep start
    double* du_ = sm.u.inc.du;
    double* dv_ = sm.u.inc.dv;
    if constexpr (kStage) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int l = C.l[k][c];
                if (l < 0) continue;
                du_[l] = s_iu[k][c];
                dv_[l] = s_iv[k][c];
            }
        }
    } else {
#pragma unroll 4
        for (int i = threadIdx.x; i < RW * RH; i += NT) {
            const int ly = i / RW, lx = i - ly * RW;
            const size_t gi = (size_t)(ry0 + ly) * W + rx0 + lx;
            du_[ly * LP + lx] = Din ? Din[gi] : 0.0;
            dv_[ly * LP + lx] = Din ? Din[n + gi] : 0.0;
        }
    }
    __syncthreads();

    // Owned increments stay in registers as well (only their owner writes
    // them), and so does the other pixel of each owned pair, which is a
    // horizontal neighbour: a half sweep reads three neighbours per plane
    // from LDS instead of five values.  An owned pixel at Chebyshev distance
    // d from the core can still reach the core's final values only while
    // d < (half sweeps left), so the sweep skips it after that: the core's
    // bits do not change, the work falls to about 40%.
    // Per owned pixel: its Chebyshev distance from the core, the LDS indices
    // of its horizontal (pair partner's other side) and vertical neighbours,
    // and whether its pair partner is to the right and inside the region.  A
    // lean tile packs them into one word (neighbours in the region: bits 0..3
    // as C.m, partner right: bit 4, partner inside: bit 5, distance: bits
    // 8..) and forms the indices in each half sweep, for registers.
    constexpr int NA = LEAN ? 1 : PPT, NP = LEAN ? PPT : 1;
    double ru[PPT][2], rv[PPT][2];
    int cd[NA][2], lh[NA][2], lvd[NA][2], lvu[NA][2];
    unsigned hs[NA][2];   // 1: pair partner to the right, 2: partner in the region
    int pk[NP][2];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int l = C.l[k][c];
            ru[k][c] = rv[k][c] = 0.0;
            if constexpr (LEAN) {
                pk[k][c] = 0;
            } else {
                cd[k][c] = 1 << 20;
                lh[k][c] = lvd[k][c] = lvu[k][c] = 0;
                hs[k][c] = 0;
            }
            if (l < 0) continue;
            ru[k][c] = du_[l];
            rv[k][c] = dv_[l];
            const int ly = l / LP, lx = l - ly * LP;
            const int x = rx0 + lx, y = ry0 + ly;
            const int d = max(max(max(cx0 - x, x - (cx1 - 1)), max(cy0 - y, y - (cy1 - 1))), 0);
            const int m = C.m[k][c];
            const bool right = (lx & 1) == 0;   // pair m covers columns 2m (partner right) and 2m + 1
            const bool pin = right ? (m & 1) : (m & 2);
            if constexpr (LEAN) {
                pk[k][c] = (m & 15) | (right ? 16 : 0) | (pin ? 32 : 0) | (d << 8);
            } else {
                cd[k][c] = d;
                lh[k][c] = right ? ((m & 2) ? l - 1 : l) : ((m & 1) ? l + 1 : l);
                lvd[k][c] = (m & 4) ? l + LP : l;
                lvu[k][c] = (m & 8) ? l - LP : l;
                hs[k][c] = (right ? 1u : 0u) | (pin ? 2u : 0u);
            }
        }
    }
    const int khe = 2 * ((kh + 1) / 2);   // half sweeps this launch runs

    // 5. red-black half sweeps: colour 0 = (x + y) even, first
    for (int j = 0; j < kh; j += 2) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int reach = khe - 1 - (j + c);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int l = C.l[k][c];
                int dist, ih, ivd, ivu;
                bool right, pin;
                if constexpr (LEAN) {
                    const int q = pk[k][c];
                    dist = q >> 8;
                    right = q & 16;
                    pin = q & 32;
                    ih = right ? ((q & 2) ? l - 1 : l) : ((q & 1) ? l + 1 : l);
                    ivd = (q & 4) ? l + LP : l;
                    ivu = (q & 8) ? l - LP : l;
                } else {
                    dist = cd[k][c];
                    right = hs[k][c] & 1u;
                    pin = hs[k][c] & 2u;
                    ih = lh[k][c];
                    ivd = lvd[k][c];
                    ivu = lvu[k][c];
                }
                if (l < 0 || dist > reach) continue;
                const double du = ru[k][c], dv = rv[k][c];
                const double pu = pin ? ru[k][c ^ 1] : du;
                const double hu = du_[ih];
                const double nu = ((C.wr[k][c] * (right ? pu : hu) + C.wl[k][c] * (right ? hu : pu)) +
                                   C.wd[k][c] * du_[ivd]) + C.wu[k][c] * du_[ivu];
                const double dun = om1 * du + C.i1[k][c] * ((nu + C.c1[k][c]) - C.a12[k][c] * dv);
                du_[l] = dun;
                ru[k][c] = dun;
                if (!stereo) {
                    const double pv = pin ? rv[k][c ^ 1] : dv;
                    const double hv = dv_[ih];
                    const double nv = ((C.wr[k][c] * (right ? pv : hv) + C.wl[k][c] * (right ? hv : pv)) +
                                       C.wd[k][c] * dv_[ivd]) + C.wu[k][c] * dv_[ivu];
                    const double dvn = om1 * dv + C.i2[k][c] * ((nv + C.c2[k][c]) - C.a12[k][c] * dun);
                    dv_[l] = dvn;
                    rv[k][c] = dvn;
                }
            }
            __syncthreads();
            if (a.tape) {
                // state after this half sweep, core pixels only (every pixel of
                // the level is the core of exactly one tile)
                auto* tp = dis_global(a.tape) + (size_t)(a.tape_m0 + j + c + 1) * 2 * n;
                const int CW = cx1 - cx0, CH = cy1 - cy0;
                for (int i = threadIdx.x; i < CW * CH; i += NT) {
                    const int yy = i / CW, xx = i - yy * CW;
                    const size_t gi = (size_t)(cy0 + yy) * W + cx0 + xx;
                    const int l = (cy0 + yy - ry0) * LP + (cx0 + xx - rx0);
                    tp[gi] = du_[l];
                    tp[n + gi] = dv_[l];
                }
                __syncthreads();   // the next half sweep rewrites what was just copied
            }
        }
    }

    // 6. the core: increment, and the refined flow after the last step
    const int CW = cx1 - cx0, CH = cy1 - cy0;
    for (int i = threadIdx.x; i < CW * CH; i += NT) {
        const int yy = i / CW, xx = i - yy * CW;
        const int x = cx0 + xx, y = cy0 + yy;
        const size_t gi = (size_t)y * W + x;
        const int l = (y - ry0) * LP + (x - rx0);
        const double du = du_[l], dv = dv_[l];
        dis_global(a.dUout)[gi] = du;
        dis_global(a.dUout)[n + gi] = dv;
        if (a.Uout) {
            double u0, v0;
            if constexpr (LEAN) {
                u0 = dis_global(a.U)[gi];
                v0 = dis_global(a.U)[n + gi];
            } else {
                u0 = sm.uu[l];
                v0 = sm.uv[l];
            }
            dis_global(a.Uout)[gi] = u0 + du;
            dis_global(a.Uout)[n + gi] = v0 + dv;
        }
    }
    __syncthreads();   // LDS is reused by the caller's next tile
}

// Phase-major launches over the same per-level tables as the persistent
// kernel: one launch per phase covers every pair (its segments are
// consecutive in the queue order), no waiting inside the launch.
template <int PS, int LPP, int NC = 1>
__global__ __launch_bounds__(256) void k_phase_search(const LevelLaunch L) {
    const int t = blockIdx.x;                       // phase 0 starts at task 0
    SearchArgs sa;
    int local = t;
    if (L.one) {
        sa = L.sa1;
    } else {
        const int j = __builtin_amdgcn_readfirstlane(L.task_seg[t]);
        sa = L.pairs[j].sa;
        local = t - __builtin_amdgcn_readfirstlane(L.start[j]);
    }
    search_block<PS, LPP, NC>(sa, local);
}

// Row-owned search (grey frames, L2 norm), one wave per block.
template <int PS, int NRB, int NH, int R>
__global__ __launch_bounds__(64) void k_phase_search_rows(const LevelLaunch L) {
    __shared__ double s_win[(64 / (NRB * NH)) * RowWin<PS, R>::SIZE];
    const int t = blockIdx.x;                       // phase 0 starts at task 0
    SearchArgs sa;
    int local = t;
    if (L.one) {
        sa = L.sa1;
    } else {
        const int j = __builtin_amdgcn_readfirstlane(L.task_seg[t]);
        sa = L.pairs[j].sa;
        local = t - __builtin_amdgcn_readfirstlane(L.start[j]);
    }
    search_rows<PS, NRB, NH, R, 64>(sa, local, s_win);
}

template <bool COLOUR = false>
__global__ __launch_bounds__(256) void k_phase_densify(const LevelLaunch L) {
    DensifyArgs da;
    int local = blockIdx.x, bx;
    if (L.one) {
        da = L.da1;
        bx = L.dens_bx1;
    } else {
        const int np = L.npairs;
        const int t = __builtin_amdgcn_readfirstlane(L.start[np]) + blockIdx.x;
        const int j = __builtin_amdgcn_readfirstlane(L.task_seg[t]) - np;
        const LevelPair& P = L.pairs[j];
        da = P.da;
        bx = P.dens_bx;
        local = t - __builtin_amdgcn_readfirstlane(L.start[np + j]);
    }
    densify_block<COLOUR>(da, local % bx, local / bx);
}

// A lean tile asks for registers that let two blocks share a CU.
template <int TW, int TH, int NT, bool COLOUR = false, bool LEAN = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(LEAN ? NT / 128 : 1)))
void k_phase_refine(const PhaseLaunch PL) {
    __shared__ RefineSmem<TW, TH, DIS_KMAX, LEAN> sm;
    const LevelLaunch& L = PL.L;
    RefineArgs ra;
    int q = dis_xcd_tile(blockIdx.x, gridDim.x), nt = gridDim.x;   // the pair's tiles, in launch order
    if (L.one) {
        ra = PL.ra1;
    } else {
        const int phase = PL.phase;
        const int np = L.npairs, s0 = phase * np;
        const int t = __builtin_amdgcn_readfirstlane(L.start[s0]) + q;
        const int j = __builtin_amdgcn_readfirstlane(L.task_seg[t]) - s0;
        ra = dis_phase_args(L.pairs[j], L.rph[phase - 2], L.lin_cache, COLOUR);
        const int t0 = __builtin_amdgcn_readfirstlane(L.start[s0 + j]);
        nt = __builtin_amdgcn_readfirstlane(L.start[s0 + j + 1]) - t0;
        q = t - t0;
    }
    refine_tile<TW, TH, NT, COLOUR, LEAN>(ra, dis_band_tile(q, ra.tiles_x, nt), sm);
}

// ----------------------------------------------------------------- upscale

// A block of the output, 256 columns by a.rows rows: each thread one
// column (every store instruction writes 64 consecutive elements).  The value
// is bilin() of each flow plane, f times.  A column's horizontal taps and
// weight are the same in every row, and a row's vertical ones are the same
// in every column; consecutive rows usually share their two source rows
// (f >= 2), so the four taps of both planes and their horizontal blends are
// formed again only when those change.  x / f is a multiplication by 1 / f,
// exact for f = 2^s.
__device__ __forceinline__ void upsample_block(const UpsArgs& a, int bx, int by) {
    const int Ws = a.Ws, Hs = a.Hs;
    const double f = a.f, inv_f = 1.0 / f;
    const double* Uu = a.U;
    const double* Uv = a.U + (size_t)Ws * Hs;
    const int xo = bx * 256 + (int)threadIdx.x;
    const int x = min(xo, a.W - 1);
    const double qx = a.centre_map ? ((double)x + 0.5) * inv_f - 0.5 : (double)x * inv_f;
    double xf = floor(qx);
    const double ax = qx - xf;
    xf = fmin(fmax(xf, -2.0), (double)Ws + 1.0);
    const int xi = (int)xf;
    const int c0 = clampi(xi, 0, Ws - 1), c1 = clampi(xi + 1, 0, Ws - 1);
    const size_t n = (size_t)a.W * a.H;
    const bool bad = a.poison && __builtin_amdgcn_readfirstlane(*dis_global(a.poison)) != 0;
    const int y0 = by * a.rows, yn = min(a.rows, a.H - y0);
    int p0 = -1, p1 = -1;
    double ut = 0.0, ub = 0.0, vt = 0.0, vb = 0.0;
    for (int i = 0; i < yn; ++i) {
        const int y = y0 + i;
        const double qy = a.centre_map ? ((double)y + 0.5) * inv_f - 0.5 : (double)y * inv_f;
        double yf = floor(qy);
        const double ay = qy - yf;
        yf = fmin(fmax(yf, -2.0), (double)Hs + 1.0);
        const int yi = (int)yf;
        const int r0 = clampi(yi, 0, Hs - 1) * Ws, r1 = clampi(yi + 1, 0, Hs - 1) * Ws;
        if (r0 != p0 || r1 != p1) {   // uniform: the rows depend on y only
            ut = (1.0 - ax) * Uu[r0 + c0] + ax * Uu[r0 + c1];
            ub = (1.0 - ax) * Uu[r1 + c0] + ax * Uu[r1 + c1];
            vt = (1.0 - ax) * Uv[r0 + c0] + ax * Uv[r0 + c1];
            vb = (1.0 - ax) * Uv[r1 + c0] + ax * Uv[r1 + c1];
            p0 = r0;
            p1 = r1;
        }
        double u = f * ((1.0 - ay) * ut + ay * ub);
        double v = f * ((1.0 - ay) * vt + ay * vb);
        if (bad) u = v = __builtin_nan("");
        if (xo >= a.W) continue;
        const size_t g = (size_t)y * a.W + xo;
        if (a.out_f64) {
            ((double*)a.out)[g] = u;
            ((double*)a.out)[n + g] = v;
        } else {
            ((float*)a.out)[g] = (float)u;
            ((float*)a.out)[n + g] = (float)v;
        }
    }
}

__global__ __launch_bounds__(256) void k_upsample(const UpsArgs a) {
    upsample_block(a, blockIdx.x, blockIdx.y);
}

// Upscaling of many pairs in one launch (blocks of pair j are start[j] ..).
__global__ __launch_bounds__(256) void k_upsample_tab(const UpsTab T) {
    const int t = blockIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(T.blk[t]);
    const UpsArgs& a = T.tab[j];
    const int local = t - __builtin_amdgcn_readfirstlane(T.start[j]);
    const int bxn = (a.W + 255) / 256;
    upsample_block(a, local % bxn, local / bxn);
}

// ------------------------------------------------- persistent level kernel

// A waiting block polls at most this many times (about a second) before it
// flags the launch as failed and moves on; with the queue's ordering a wait
// always ends long before that.
constexpr int kSpinLimit = 1 << 21;

// A whole pair-level in one 1024-thread block (Sec. 2.2 step 3 and Sec. 2.3
// for levels of at most DIS_SMALL_PAIRS pixel pairs): densification into
// LDS, then every fixed-point step with its red-black sweeps on the whole
// level, no tiles and no halo.  Each thread owns one horizontal pixel pair
// (one pixel of each colour), as in the tiled kernel, and does the same
// arithmetic in the same order, so the result is the tiled one bit for bit.
struct SmallSmem {
    double J0[DIS_SMALL_PX], J1w[DIS_SMALL_PX];
    double uu[DIS_SMALL_PX], uv[DIS_SMALL_PX];
    double du[DIS_SMALL_PX], dv[DIS_SMALL_PX];
    double wr[DIS_SMALL_PX], wd[DIS_SMALL_PX];
};

template <int NT, int PPT>
__device__ __forceinline__ void small_level(const DensifyArgs& da, const RefineArgs& a, int nouter_, int nhalf_,
                                            SmallSmem& sm) {
    // J0 and the warped J1 stay fixed for the whole level, so with one pair
    // per thread and registers to spare the linearisation of the owned
    // pixels (derivatives and their normalisations, Sec. 2.3) is computed
    // once, before the fixed-point steps
    constexpr bool kLinReg = PPT == 1 && NT <= 512;
    const int W = a.W, H = a.H;
    const int npx = W * H;
    const size_t n = (size_t)npx;

    // 1. densification, the warped second frame, J0
    for (int i = threadIdx.x; i < npx; i += NT) {
        const int y = i / W, x = i - y * W;
        double U, V, sw;
        densify_pixel(da, x, y, U, V, sw);
        const double jw = bilin(da.J1, W, H, (double)x + U, (double)y + V);
        if (da.Z) da.Z[i] = sw;
        da.U[i] = U;
        da.U[n + i] = V;
        da.J1w[i] = jw;
        sm.uu[i] = U;
        sm.uv[i] = V;
        sm.J1w[i] = jw;
        sm.J0[i] = a.J0[i];
        sm.du[i] = 0.0;
        sm.dv[i] = 0.0;
    }
    __syncthreads();

    // owned pairs pr = thread + k NT: row ly, pair m; colour c at column
    // 2m + ((y & 1) ^ c)
    const int npw = (W + 1) / 2;
    int c_l[PPT][2];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pr = threadIdx.x + k * NT;
        const int ly = pr / npw, m = pr - ly * npw;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int lx = 2 * m + ((ly & 1) ^ c);
            c_l[k][c] = (pr < npw * H && lx < W) ? ly * W + lx : -1;
        }
    }
    const double om = a.omega, om1 = 1.0 - a.omega;
    const double eps2 = a.eps * a.eps;
    const int nouter = __builtin_amdgcn_readfirstlane(nouter_);
    const int nhalf = __builtin_amdgcn_readfirstlane(nhalf_);
    auto Ib = [&](int x, int y) { const int l = y * W + x; return 0.5 * (sm.J0[l] + sm.J1w[l]); };
    auto Ixa = [&](int x, int y) { return (Ib(min(x + 1, W - 1), y) - Ib(max(x - 1, 0), y)) / 2.0; };
    auto Iya = [&](int x, int y) { return (Ib(x, min(y + 1, H - 1)) - Ib(x, max(y - 1, 0))) / 2.0; };
    // Ix, Iy, Iz, Ixx, Ixy, Iyy, Ixz, Iyz, b0, bx, by of pixel l = (x, y)
    auto linearise = [&](int l, int x, int y, double (&q)[11]) {
        const int xm = max(x - 1, 0), xp = min(x + 1, W - 1);
        const int ym = max(y - 1, 0), yp = min(y + 1, H - 1);
        const double* t0 = sm.J0;
        const double* t1 = sm.J1w;
        const double Ix = Ixa(x, y), Iy = Iya(x, y);
        const double Ixx = (Ixa(xp, y) - Ixa(xm, y)) / 2.0;
        const double Ixy = (Ixa(x, yp) - Ixa(x, ym)) / 2.0;
        const double Iyy = (Iya(x, yp) - Iya(x, ym)) / 2.0;
        const int lxp = y * W + xp, lxm = y * W + xm, lyp = yp * W + x, lym = ym * W + x;
        q[0] = Ix;
        q[1] = Iy;
        q[2] = t1[l] - t0[l];
        q[3] = Ixx;
        q[4] = Ixy;
        q[5] = Iyy;
        q[6] = (t1[lxp] - t1[lxm]) / 2.0 - (t0[lxp] - t0[lxm]) / 2.0;
        q[7] = (t1[lyp] - t1[lym]) / 2.0 - (t0[lyp] - t0[lym]) / 2.0;
        q[8] = 1.0 / ((Ix * Ix + Iy * Iy) + 0.01);
        q[9] = 1.0 / ((Ixx * Ixx + Ixy * Ixy) + 0.01);
        q[10] = 1.0 / ((Ixy * Ixy + Iyy * Iyy) + 0.01);
    };
    double r_u[PPT][2], r_v[PPT][2];   // the owned increments (zero at the start of the level)
#pragma unroll
    for (int k = 0; k < PPT; ++k)
#pragma unroll
        for (int c = 0; c < 2; ++c) r_u[k][c] = r_v[k][c] = 0.0;
    double lin_r[kLinReg ? 2 : 1][11];
    if constexpr (kLinReg) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int l = c_l[0][c];
            if (l < 0) continue;
            const int y = l / W, x = l - y * W;
            linearise(l, x, y, lin_r[c]);
        }
    }

    for (int it = 0; it < nouter; ++it) {
        // the owned positions, re-derived each step: otherwise the compiler
        // hoists every neighbour address of the step out of the loop and
        // spills them (an empty asm makes the copy opaque)
        int cl[PPT][2];
#pragma unroll
        for (int k = 0; k < PPT; ++k)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                int v = c_l[k][c];
                __asm__ volatile("" : "+v"(v));
                cl[k][c] = v;
            }
        // 2. smoothness weights from U + dU (the frozen increment is the
        //    current one: the whole level is here)
        double c_ws[PPT][2];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                c_ws[k][c] = 0.0;
                const int e = cl[k][c];
                if (e < 0) continue;
                const int y = e / W, x = e - y * W;
                const double u0 = sm.uu[e] + sm.du[e], v0 = sm.uv[e] + sm.dv[e];
                double dxu = 0.0, dyu = 0.0, dxv = 0.0, dyv = 0.0;
                if (x < W - 1) {
                    dxu = (sm.uu[e + 1] + sm.du[e + 1]) - u0;
                    dxv = (sm.uv[e + 1] + sm.dv[e + 1]) - v0;
                }
                if (y < H - 1) {
                    dyu = (sm.uu[e + W] + sm.du[e + W]) - u0;
                    dyv = (sm.uv[e + W] + sm.dv[e + W]) - v0;
                }
                const double es = ((dxu * dxu + dyu * dyu) + dxv * dxv) + dyv * dyv;
                c_ws[k][c] = a.alpha / (2.0 * sqrt(es + eps2));
            }
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int e = cl[k][c];
                if (e < 0) continue;
                const int y = e / W, x = e - y * W;
                sm.wr[e] = x < W - 1 ? c_ws[k][c] : 0.0;
                sm.wd[e] = y < H - 1 ? c_ws[k][c] : 0.0;
            }
        }
        __syncthreads();
        // 3. coefficients of the owned pixels
        int c_m[PPT][2];
        double c_wr[PPT][2], c_wl[PPT][2], c_wd[PPT][2], c_wu[PPT][2];
        double c_a12[PPT][2], c_i1[PPT][2], c_i2[PPT][2], c_c1[PPT][2], c_c2[PPT][2];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                c_m[k][c] = 0;
                c_wr[k][c] = c_wl[k][c] = c_wd[k][c] = c_wu[k][c] = 0.0;
                c_a12[k][c] = c_i1[k][c] = c_i2[k][c] = c_c1[k][c] = c_c2[k][c] = 0.0;
                const int l = cl[k][c];
                if (l < 0) continue;
                const int y = l / W, x = l - y * W;
                double q[11];
                if constexpr (kLinReg) {
#pragma unroll
                    for (int i = 0; i < 11; ++i) q[i] = lin_r[c][i];
                } else {
                    linearise(l, x, y, q);
                }
                const double Ix = q[0], Iy = q[1], Iz = q[2], Ixx = q[3], Ixy = q[4], Iyy = q[5];
                const double Ixz = q[6], Iyz = q[7], b0 = q[8], bx = q[9], by = q[10];
                const double fu = it ? sm.du[l] : 0.0, fv = it ? sm.dv[l] : 0.0;
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
                const bool hr = x < W - 1, hl = x > 0, hd = y < H - 1, hu = y > 0;
                const double wr = hr ? sm.wr[l] : 0.0, wl = hl ? sm.wr[l - 1] : 0.0;
                const double wd = hd ? sm.wd[l] : 0.0, wu = hu ? sm.wd[l - W] : 0.0;
                const double Ssum = ((wr + wl) + wd) + wu;
                const double Up = sm.uu[l], Vp = sm.uv[l];
                const double Ur = hr ? sm.uu[l + 1] : 0.0, Ul = hl ? sm.uu[l - 1] : 0.0;
                const double Ud = hd ? sm.uu[l + W] : 0.0, Uu = hu ? sm.uu[l - W] : 0.0;
                const double Vr = hr ? sm.uv[l + 1] : 0.0, Vl = hl ? sm.uv[l - 1] : 0.0;
                const double Vd = hd ? sm.uv[l + W] : 0.0, Vu = hu ? sm.uv[l - W] : 0.0;
                const double NU = ((wr * Ur + wl * Ul) + wd * Ud) + wu * Uu;
                const double NV = ((wr * Vr + wl * Vl) + wd * Vd) + wu * Vu;
                // 16: the pair's other pixel (columns 2m, 2m + 1) is to the right;
                // 32: it exists
                const bool rt = (x & 1) == 0;
                c_m[k][c] = (hr ? 1 : 0) | (hl ? 2 : 0) | (hd ? 4 : 0) | (hu ? 8 : 0) | (rt ? 16 : 0) |
                            ((rt ? hr : hl) ? 32 : 0);
                c_wr[k][c] = wr; c_wl[k][c] = wl; c_wd[k][c] = wd; c_wu[k][c] = wu;
                c_a12[k][c] = A12;
                c_i1[k][c] = om / (A11 + Ssum);
                c_i2[k][c] = om / (A22 + Ssum);
                c_c1[k][c] = (NU - Ssum * Up) - B1;
                c_c2[k][c] = (NV - Ssum * Vp) - B2;
                __builtin_amdgcn_sched_barrier(0);   // one pixel's temporaries at a time
            }
        }
        __syncthreads();   // every frozen increment is read before the sweeps move it
        // 4. red-black half sweeps: colour 0 = (x + y) even, first
        for (int jh = 0; jh < nhalf; jh += 2) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const int l = cl[k][c];
                    if (l < 0) continue;
                    // with registers to spare, the owned increments and the
                    // pair's other pixel come from registers (only this
                    // thread writes them), three neighbours per plane from LDS
                    const int m = c_m[k][c];
                    const bool right = m & 16, pin = m & 32;
                    const int lh = right ? ((m & 2) ? l - 1 : l) : ((m & 1) ? l + 1 : l);
                    const int ld = (m & 4) ? l + W : l, lu = (m & 8) ? l - W : l;
                    const int lp = right ? l + 1 : l - 1;   // the pair's other pixel
                    const double du = kLinReg ? r_u[k][c] : sm.du[l], dv = kLinReg ? r_v[k][c] : sm.dv[l];
                    const double pu = pin ? (kLinReg ? r_u[k][c ^ 1] : sm.du[lp]) : du;
                    const double hu_ = sm.du[lh];
                    const double nu = ((c_wr[k][c] * (right ? pu : hu_) + c_wl[k][c] * (right ? hu_ : pu)) +
                                       c_wd[k][c] * sm.du[ld]) + c_wu[k][c] * sm.du[lu];
                    const double dun = om1 * du + c_i1[k][c] * ((nu + c_c1[k][c]) - c_a12[k][c] * dv);
                    sm.du[l] = dun;
                    r_u[k][c] = dun;
                    if (!a.stereo) {
                        const double pv = pin ? (kLinReg ? r_v[k][c ^ 1] : sm.dv[lp]) : dv;
                        const double hv_ = sm.dv[lh];
                        const double nv = ((c_wr[k][c] * (right ? pv : hv_) + c_wl[k][c] * (right ? hv_ : pv)) +
                                           c_wd[k][c] * sm.dv[ld]) + c_wu[k][c] * sm.dv[lu];
                        const double dvn = om1 * dv + c_i2[k][c] * ((nv + c_c2[k][c]) - c_a12[k][c] * dun);
                        sm.dv[l] = dvn;
                        r_v[k][c] = dvn;
                    }
                }
                __syncthreads();
            }
        }
        // (the next step's first reads follow the last half sweep's barrier)
    }
    // 5. refined flow
    for (int i = threadIdx.x; i < npx; i += NT) {
        a.Uout[i] = sm.uu[i] + sm.du[i];
        a.Uout[n + i] = sm.uv[i] + sm.dv[i];
    }
}

// ONE: a single pair, whose arguments the launch carries (read in place);
// else block b takes pairs[list[b]].  One pixel pair per thread: 512
// threads serve levels of at most 512 pairs, 1024 threads the rest; the
// narrower block has twice the registers per thread, enough to keep the
// linearisation.
template <int NT, bool ONE>
__global__ __launch_bounds__(NT) void k_small_level(const SmallLaunch S) {
    static_assert(NT == 512 || NT == DIS_SMALL_PAIRS, "one pixel pair per thread, up to the LDS capacity");
    __shared__ SmallSmem sm;
    if constexpr (ONE) {
        small_level<NT, 1>(S.da1, S.ra1, S.nouter, S.nhalf, sm);
    } else {
        const LevelPair& P = S.pairs[__builtin_amdgcn_readfirstlane(S.list[blockIdx.x])];
        small_level<NT, 1>(P.da, P.ra, S.nouter, S.nhalf, sm);
    }
}

// Queue operations of thread 0.  They are kept out of line on purpose: the
// level kernel's loop holds barriers, and with these thread-0 branches
// inlined at the loop's edges the compiler's control-flow structurisation
// can let the other threads run ahead into the next iteration's barrier.
// Out of line, the loop body the compiler sees is uniform.
__device__ __attribute__((noinline)) void lane0_take(int* head, int* s_task) {
    if (threadIdx.x == 0) *s_task = __hip_atomic_fetch_add(head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A wait that gives up marks its launch (err) and the whole plan (plan_err):
// the task is skipped, and the upscaling then writes the plan's flows as NaN,
// so a failed wait cannot pass as a result.  `give_up` makes every wait on
// a predecessor fail at once (the host forces it to test this path; every
// kernel still runs to its end).
__device__ __attribute__((noinline)) void lane0_wait(const int* ctr, int need, int* err, int* plan_err, int give_up,
                                                     int* s_ok) {
    if (threadIdx.x == 0) {
        int ok = 1, spins = 0;
        if (give_up && need > 0) {
            ok = 0;
        } else {
            while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
                if (++spins > kSpinLimit) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        if (!ok) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (plan_err) __hip_atomic_store(plan_err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        *s_ok = ok;
    }
}

__device__ __attribute__((noinline)) void lane0_signal(int* ctr, int n) {
    if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Every pair's work at one level as one launch.  Blocks take tasks from the
// queue in order; a task of phase p of pair j first waits until phase p-1 of
// pair j has finished (all those tasks were taken earlier, by running blocks).
// RNRB > 0: the search is the row-owned one (layout RNRB x RNH, window
// radius RR), whose windows share LDS with the refinement tile.
// TW x TH: the refinement core of the level's tiles (on 256 threads, as
// every task of the launch)
template <int PS, int LPP, int RNRB = 0, int RNH = 0, int RR = 0, int TW = 32, int TH = 16>
__global__ __launch_bounds__(256) void k_level(const LevelLaunch L) {
    constexpr int WIN = RNRB > 0 ? (256 / LPP) * RowWin<PS, RR>::SIZE : 1;
    __shared__ union LevelSmem {
        RefineSmem<TW, TH> r;
        double win[WIN];
    } smu;
    RefineSmem<TW, TH>& sm = smu.r;
    __shared__ int s_task, s_ok;
    int* head = L.sync;
    int* err = L.sync + 1;
    int* done = L.sync + 2;
    // every value steering this loop is made wave-uniform explicitly
    for (;;) {
        lane0_take(head, &s_task);
        __syncthreads();
        const int r = __builtin_amdgcn_readfirstlane(s_task);
        __syncthreads();   // s_task is rewritten on the next round
        if (r >= L.nruns) break;
        const int t0 = __builtin_amdgcn_readfirstlane(L.run_start[r]);
        const int t1 = __builtin_amdgcn_readfirstlane(L.run_start[r + 1]);
        const int seg = __builtin_amdgcn_readfirstlane(L.task_seg[t0]);
        const int phase = seg / L.npairs, pair = seg - phase * L.npairs;
        const int first = __builtin_amdgcn_readfirstlane(L.start[seg]);
        const int prev = phase > 0 ? seg - L.npairs : seg;
        const int need = phase > 0 ? __builtin_amdgcn_readfirstlane(L.start[prev + 1] - L.start[prev]) : 0;
        lane0_wait(done + prev, need, err, L.plan_err, L.fail_waits, &s_ok);
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int ok = __builtin_amdgcn_readfirstlane(s_ok);
        const LevelPair& P = L.pairs[pair];
        for (int t = t0; t < t1 && ok; ++t) {
            const int local = t - first;
            if (phase == 0) {
                if constexpr (RNRB > 0) search_rows<PS, RNRB, RNH, RR, 256>(P.sa, local, smu.win);
                else search_block<PS, LPP>(P.sa, local);
            } else if (phase == 1) {
                densify_block(P.da, local % P.dens_bx, local / P.dens_bx);
            } else {
                RefineArgs ra = dis_phase_args(P, L.rph[phase - 2], L.lin_cache, false);
                ra.nhalf = __builtin_amdgcn_readfirstlane(ra.nhalf);
                refine_tile<TW, TH, 256>(ra, local, sm);
            }
            __syncthreads();   // LDS (windows, tile) is reused by the run's next task
        }
        __threadfence();
        __syncthreads();
        lane0_signal(done + seg, t1 - t0);
    }
}

}  // namespace

// ------------------------------------------------------------ kernel table

const void* dis_kernel_pyramid() { return (const void*)&k_pyramid; }
const void* dis_kernel_pyramid_tab() { return (const void*)&k_pyramid_tab; }
const void* dis_kernel_upsample() { return (const void*)&k_upsample; }
const void* dis_kernel_upsample_tab() { return (const void*)&k_upsample_tab; }
const void* dis_kernel_phase_densify() { return (const void*)&k_phase_densify<false>; }
const void* dis_kernel_phase_densify_colour() { return (const void*)&k_phase_densify<true>; }
const void* dis_kernel_small_level(int threads, bool one) {
    if (threads == 512) return one ? (const void*)&k_small_level<512, true> : (const void*)&k_small_level<512, false>;
    if (threads == 1024) return one ? (const void*)&k_small_level<1024, true> : (const void*)&k_small_level<1024, false>;
    return nullptr;
}
const void* dis_kernel_fb_count() { return (const void*)&k_fb_count; }
const void* dis_kernel_fb_scan() { return (const void*)&k_fb_scan; }
const void* dis_kernel_fb_scatter() { return (const void*)&k_fb_scatter; }
const void* dis_kernel_fb_densify() { return (const void*)&k_fb_densify; }
const void* dis_kernel_colour_lin() { return (const void*)&k_colour_lin; }

// colour search instances: 32 lanes per patch (16 below 8x8 patches) keep
// the three channels' per-lane pixel arrays within the register file
int dis_colour_lanes(int ps) { return ps < 8 ? 16 : 32; }

const void* dis_kernel_phase_search_colour(int ps) {
    switch (ps) {
        case 4: return (const void*)&k_phase_search<4, 16, 3>;
        case 6: return (const void*)&k_phase_search<6, 16, 3>;
        case 8: return (const void*)&k_phase_search<8, 32, 3>;
        case 10: return (const void*)&k_phase_search<10, 32, 3>;
        case 12: return (const void*)&k_phase_search<12, 32, 3>;
        default: return nullptr;
    }
}

// instances whose per-lane pixel arrays fit the 256 architectural VGPRs
#define DIS_FOR_SEARCH_INSTANCES(X) \
    X(4, 4) X(4, 8) X(4, 16) X(6, 4) X(6, 8) X(6, 16) X(8, 4) X(8, 8) X(8, 16) X(8, 32) X(8, 64) \
    X(10, 8) X(10, 16) X(10, 32) X(10, 64) X(12, 8) X(12, 16) X(12, 32) X(12, 64) X(14, 16) X(14, 32) \
    X(14, 64) X(16, 16) X(16, 32) X(16, 64)

#define DIS_SEARCH_CASE(PS_, LPP_) \
    if (ps == PS_ && lpp == LPP_) return (const void*)&k_phase_search<PS_, LPP_>;
#define DIS_LEVEL_CASE(PS_, LPP_) \
    if (ps == PS_ && lpp == LPP_) return (const void*)&k_level<PS_, LPP_>;

const void* dis_kernel_phase_search(int ps, int lpp) {
    DIS_FOR_SEARCH_INSTANCES(DIS_SEARCH_CASE)
    return nullptr;
}

const void* dis_kernel_level(int ps, int lpp) {
    DIS_FOR_SEARCH_INSTANCES(DIS_LEVEL_CASE)
    return nullptr;
}

// row-owned search layouts (patch size, row blocks, column halves, window
// radius): lanes per patch = row blocks x halves
#define DIS_FOR_ROW_INSTANCES(X) \
    X(4, 4, 1, 3) X(4, 4, 2, 3) X(6, 2, 1, 3) X(6, 2, 2, 3) X(8, 4, 1, 3) X(8, 4, 2, 3) X(8, 8, 2, 3) \
    X(10, 2, 2, 2) X(12, 2, 2, 2) X(12, 4, 2, 2) X(16, 4, 2, 2) X(16, 8, 2, 2)

const void* dis_kernel_phase_search_rows(int ps, int lpp) {
#define DIS_ROWS_CASE(PS_, NRB_, NH_, R_) \
    if (ps == PS_ && lpp == NRB_ * NH_) return (const void*)&k_phase_search_rows<PS_, NRB_, NH_, R_>;
    DIS_FOR_ROW_INSTANCES(DIS_ROWS_CASE)
#undef DIS_ROWS_CASE
    return nullptr;
}

// inside the 256-thread level kernel the windows of 256 / lpp patches share
// LDS with the refinement tile: the radius shrinks until they fit 96 KB (the
// radius never changes a result, only how often a window is reloaded)
constexpr int dis_level_win_r(int ps, int lpp, int r) {
    return (r > 0 && (256 / lpp) * (ps + 1 + 2 * r) * (ps + 1 + 2 * r) * 8 > 96 * 1024) ? dis_level_win_r(ps, lpp, r - 1)
                                                                                       : r;
}

const void* dis_kernel_level_rows(int ps, int lpp, int tile) {
#define DIS_ROWS_LEVEL_CASE(PS_, NRB_, NH_, R_)                                                                    \
    if (ps == PS_ && lpp == NRB_ * NH_)                                                                            \
        return tile == 1 ? (const void*)&k_level<PS_, NRB_ * NH_, NRB_, NH_, dis_level_win_r(PS_, NRB_ * NH_, R_), \
                                                 16, 16>                                                           \
                         : (const void*)&k_level<PS_, NRB_ * NH_, NRB_, NH_, dis_level_win_r(PS_, NRB_ * NH_, R_)>;
    DIS_FOR_ROW_INSTANCES(DIS_ROWS_LEVEL_CASE)
#undef DIS_ROWS_LEVEL_CASE
    return nullptr;
}

// refinement tile shapes: core width, height, threads per block, lean (no
// LDS copy of U, two blocks per CU)
#define DIS_FOR_REFINE_TILES(X) \
    X(0, 32, 16, 256, false) X(1, 16, 16, 256, false) X(2, 64, 8, 256, false) X(3, 16, 16, 1024, false) \
    X(4, 32, 16, 1024, false) X(5, 16, 16, 512, false) X(6, 32, 16, 512, false) X(7, 8, 8, 512, false) \
    X(8, 16, 8, 512, false) X(9, 8, 8, 256, false) X(10, 8, 4, 384, false) X(11, 32, 16, 512, true) \
    X(12, 16, 16, 512, true)

int dis_refine_tile(int tile, int* tw, int* th, int* nt) {
#define DIS_TILE_SHAPE(ID, TW_, TH_, NT_, LEAN_) \
    if (tile == ID) { *tw = TW_; *th = TH_; if (nt) *nt = NT_; return 1; }
    DIS_FOR_REFINE_TILES(DIS_TILE_SHAPE)
#undef DIS_TILE_SHAPE
    return 0;
}

int dis_refine_tile_lean(int tile) {
    int tw, th, nt;
    if (!dis_refine_tile(tile, &tw, &th, &nt)) return -1;
#define DIS_TILE_TWIN(ID, TW_, TH_, NT_, LEAN_) \
    if (LEAN_ && TW_ == tw && TH_ == th && NT_ == nt) return ID;
    DIS_FOR_REFINE_TILES(DIS_TILE_TWIN)
#undef DIS_TILE_TWIN
    return -1;
}

const void* dis_kernel_phase_refine(int tile) {
#define DIS_TILE_KERNEL(ID, TW_, TH_, NT_, LEAN_) \
    if (tile == ID) return (const void*)&k_phase_refine<TW_, TH_, NT_, false, LEAN_>;
    DIS_FOR_REFINE_TILES(DIS_TILE_KERNEL)
#undef DIS_TILE_KERNEL
    return nullptr;
}

const void* dis_kernel_phase_refine_colour(int tile) {
#define DIS_TILE_KERNEL(ID, TW_, TH_, NT_, LEAN_) \
    if (tile == ID) return (const void*)&k_phase_refine<TW_, TH_, NT_, true, LEAN_>;
    DIS_FOR_REFINE_TILES(DIS_TILE_KERNEL)
#undef DIS_TILE_KERNEL
    return nullptr;
}
