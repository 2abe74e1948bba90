// Inverse search with row-owned lanes: the grey, least-squares form of the
// patch search (Sec. 2.1 and Suppl. A; stereo of App. I), included by
// dis_kernels.hip after its helpers (clampi, dis_global) and the lane moves.
//
// A patch of PS x PS pixels is split between LPP = NRB * NH lanes: NRB
// blocks of RB = PS / NRB consecutive rows times NH (1 or 2) column halves
// of CB = PS / NH columns.  Because a lane holds whole (half) rows, the
// bilinear warp at x + u is separable with one fractional offset per patch:
// each row of taps is interpolated horizontally once and shared by the two
// pixel rows it lies between, so a lane reads (RB + 1) (CB + 1) taps for its
// RB CB pixels (1.6 per pixel at 12 x 12 on 8 lanes, against 4 for
// independent pixels).
//
// Every patch sum has one canonical order, the same for all layouts:
//   S = S_left + S_right over the two column halves, where
//   S_half = a binary tree over the G = PS / RG row groups (RG = PS over the
//            largest power of two dividing it: G is a power of two), and a
//            group's value is its rows' half-row sums added in row order,
//            each half-row summed left to right (products: the first a
//            product, then fused multiply-adds).
// A lane holds whole aligned subtrees of that tree (RB is RG times a power
// of two), the lanes of a patch are numbered half-major (l = h NRB + rb), so
// the lane butterfly pairs row blocks of one half first and the halves last:
// every layout, and so every lanes-per-patch choice, gives the same bits.
//
// The right-hand side uses sum g (d - mean d) = sum (g - mean g) Q -
// sum (g - mean g) T, with g the template gradient, Q = I1(x + u) and
// d = Q - T: the centred gradients and the template term are formed once per
// patch, and each iteration needs two sums of products with Q, not three
// sums.
#pragma once
#include <type_traits>

constexpr int dis_largest_pow2_divisor(int v) { return v % 2 == 0 ? 2 * dis_largest_pow2_divisor(v / 2) : 1; }

template <int PS, int NRB_, int NH_>
struct RowLayout {
    static constexpr int NH = NH_;
    static constexpr int NRB = NRB_;
    static constexpr int G = dis_largest_pow2_divisor(PS);   // row groups
    static constexpr int RG = PS / G;                          // rows per group
    static constexpr int RB = PS / NRB_;                       // rows per lane
    static constexpr int CB = PS / NH_;                        // columns per lane
    static constexpr int LPP = NRB_ * NH_;
    static constexpr int GPL = RB / RG;                        // groups per lane
    static_assert(NH_ == 1 || NH_ == 2, "whole rows or halves");
    static_assert(PS % 2 == 0, "even patch sizes");
    static_assert(G % NRB_ == 0, "a row block holds whole groups");
    static_assert((GPL & (GPL - 1)) == 0, "a lane holds an aligned subtree of groups");
    static_assert(LPP <= 16, "the lanes of a patch sit in one row of 16 lanes");
};

// Canonical partial sums of a lane for M values at once.  v[m][r][c] are the
// lane's pixels (rows r < RB, columns c < CB of its block).  PROD: the values
// are products a[m] * b (b shared).  Returns the lane's subtree value of each
// column half it holds: out[m][0] (left or its only half), out[m][1] (right,
// only for NH == 1).
template <class L, int M, bool PROD>
__device__ __forceinline__ void rows_partial(double (*a)[L::RB][L::CB], double (&b)[L::RB][L::CB],
                                             double (&out)[M][2]) {
    constexpr int HALVES = L::NH == 1 ? 2 : 1;
    constexpr int HC = L::CB / HALVES;     // columns per half in this lane
#pragma unroll
    for (int hh = 0; hh < HALVES; ++hh) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            double grp[L::GPL];
#pragma unroll
            for (int g = 0; g < L::GPL; ++g) {
                double acc = 0.0;
#pragma unroll
                for (int rr = 0; rr < L::RG; ++rr) {
                    const int r = g * L::RG + rr;
                    double s;
                    if constexpr (PROD) {
                        s = a[m][r][hh * HC] * b[r][hh * HC];
#pragma unroll
                        for (int c = 1; c < HC; ++c) s = fma(a[m][r][hh * HC + c], b[r][hh * HC + c], s);
                    } else {
                        s = a[m][r][hh * HC];
#pragma unroll
                        for (int c = 1; c < HC; ++c) s = s + a[m][r][hh * HC + c];
                    }
                    acc = rr == 0 ? s : acc + s;
                }
                grp[g] = acc;
            }
#pragma unroll
            for (int step = 1; step < L::GPL; step <<= 1)
#pragma unroll
                for (int g = 0; g < L::GPL; g += 2 * step) grp[g] = grp[g] + grp[g + step];
            out[m][hh] = grp[0];
        }
    }
}

// Finish the canonical sums across the LPP lanes of each patch (every lane
// of the patch receives them).
template <class L, int M>
__device__ __forceinline__ void rows_finish(double (&part)[M][2], double (&s)[M]) {
    if constexpr (L::NH == 2) {
#pragma unroll
        for (int m = 0; m < M; ++m) s[m] = lane_sum<L::LPP>(part[m][0]);
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m) s[m] = lane_sum<L::LPP>(part[m][0]) + lane_sum<L::LPP>(part[m][1]);
    }
}

// Window of the second frame kept in LDS per patch: (PS + 1 + 2R)^2 taps
// around the patch's current integer displacement (indices clamped to the
// image as the bilinear taps clamp them).  When the displacement leaves the
// window the patch reloads it around its new position, so every warp reads
// LDS.
template <int PS, int R>
struct RowWin {
    static constexpr int WS = PS + 1 + 2 * R;
    static constexpr int PITCH = WS | 1;     // odd row pitch in doubles: consecutive rows start in other banks
    static constexpr int SIZE = WS * PITCH;
};

template <int PS, int NRB, int NH, int R, int LPP>
__device__ __forceinline__ void rows_window_fill(double* win, const double* __restrict__ J1, int W, int H, int wx, int wy,
                                                 int lane) {
    using RW = RowWin<PS, R>;
    constexpr int N = RW::WS * RW::WS;
    constexpr int PER = (N + LPP - 1) / LPP;
    constexpr int HALF = (PER + 1) / 2;
    // two rounds, each issuing all its loads before its stores
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        double v[HALF];
#pragma unroll
        for (int k = 0; k < HALF; ++k) {
            const int i = lane + (part * HALF + k) * LPP;
            const int Y = i / RW::WS, X = i - Y * RW::WS;
            v[k] = i < N ? dis_global(J1)[clampi(wy + Y, 0, H - 1) * W + clampi(wx + X, 0, W - 1)] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < HALF; ++k) {
            const int i = lane + (part * HALF + k) * LPP;
            const int Y = i / RW::WS, X = i - Y * RW::WS;
            if (i < N) win[Y * RW::PITCH + X] = v[k];
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// One block of NT threads = NT / LPP patches, each with a window of
// RowWin<PS, R>::SIZE doubles at s_win (NT / LPP of them).  Same steps and outputs as
// search_block for one channel and the L2 norm: patch corner, initialisation
// from the coarser flow (Sec. 2.2 steps 1-2), template and Sobel/8
// gradients, H' = sum g g^T + lambda I, theta_it updates
// u <- u - H'^-1 sum g r with r the mean-normalised residual, the reset test,
// and the mean residual at the final u.
template <int PS, int NRB, int NH, int R, int NT>
__device__ __forceinline__ void search_rows(const SearchArgs& a, int block, double* s_win) {
    using L = RowLayout<PS, NRB, NH>;
    using RW = RowWin<PS, R>;
    constexpr int LPP = L::LPP, RB = L::RB, CB = L::CB;
    const int W = a.W, H = a.H;
    const int lane = threadIdx.x & (LPP - 1);
    const int hh = lane / NRB, rb = lane - hh * NRB;
    const int r0 = rb * RB, c0 = hh * CB;       // the lane's block inside the patch
    const int N = a.nx * a.ny;
    int pi = (int)((block * (unsigned)NT + threadIdx.x) / LPP);
    const bool valid = pi < N;
    if (!valid) pi = N - 1;    // idle lanes shadow the last patch (no store): DPP stays uniform

    const int ky = pi / a.nx, kx = pi - ky * a.nx;
    const int x0 = kx < a.nrx ? kx * a.st : W - PS;
    const int y0 = ky < a.nry ? ky * a.st : H - PS;

    // coarser-flow taps at the patch centre (bilin() of U_{s+1}, times 2)
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
        const int cc0 = clampi(xi, 0, Wn - 1), cc1 = clampi(xi + 1, 0, Wn - 1);
        const int rr0 = clampi(yi, 0, Hn - 1) * Wn, rr1 = clampi(yi + 1, 0, Hn - 1) * Wn;
        const auto* Vp = Up + (has_un ? (size_t)Wn * Hn : 0);
        u00 = Up[rr0 + cc0]; u01 = Up[rr0 + cc1]; u10 = Up[rr1 + cc0]; u11 = Up[rr1 + cc1];
        v00 = Vp[rr0 + cc0]; v01 = Vp[rr0 + cc1]; v10 = Vp[rr1 + cc0]; v11 = Vp[rr1 + cc1];
    }

    // template and Sobel/8 gradients of the lane's pixels (replicated
    // border): the lane's block and a one-pixel ring, each tap loaded once
    double T[RB][CB], gx[RB][CB], gy[RB][CB];
    {
        const auto* __restrict__ J0 = dis_global(a.J0);
        double b[RB + 2][CB + 2];
#pragma unroll
        for (int r = 0; r < RB + 2; ++r) {
            const int y = clampi(y0 + r0 + r - 1, 0, H - 1);
#pragma unroll
            for (int c = 0; c < CB + 2; ++c) b[r][c] = J0[y * W + clampi(x0 + c0 + c - 1, 0, W - 1)];
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                T[r][c] = b[r + 1][c + 1];
                const double dm = b[r][c + 2] - b[r][c];
                const double d0 = b[r + 1][c + 2] - b[r + 1][c];
                const double dp = b[r + 2][c + 2] - b[r + 2][c];
                gx[r][c] = ((dm + 2.0 * d0) + dp) / 8.0;
                const double em = b[r + 2][c] - b[r][c];
                const double e0 = b[r + 2][c + 1] - b[r][c + 1];
                const double ep = b[r + 2][c + 2] - b[r][c + 2];
                gy[r][c] = ((em + 2.0 * e0) + ep) / 8.0;
            }
        }
    }
    // H' and the gradient sums, five canonical sums in one tree pass
    double h11, h12, h22, mgx, mgy;
    {
        double src[2][RB][CB];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < CB; ++c) { src[0][r][c] = gx[r][c]; src[1][r][c] = gy[r][c]; }
        double pa[2][2], pb[1][2], pc[2][2];
        rows_partial<L, 2, true>(src, gx, pa);          // sum gx gx, sum gy gx
        rows_partial<L, 1, true>(&src[1], gy, pb);      // sum gy gy
        rows_partial<L, 2, false>(src, gx, pc);         // sum gx, sum gy
        double p5[5][2], s5[5];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            p5[0][k] = pa[0][k]; p5[1][k] = pa[1][k]; p5[2][k] = pb[0][k];
            p5[3][k] = pc[0][k]; p5[4][k] = pc[1][k];
        }
        rows_finish<L, 5>(p5, s5);
        h11 = s5[0]; h12 = s5[1]; h22 = s5[2];
        mgx = s5[3] / (double)(PS * PS);
        mgy = s5[4] / (double)(PS * PS);
    }
    // centred gradients: sum g (d - mean d) == sum (g - mean g) d, and with
    // d = Q - T that is sum (g - mean g) Q - sum (g - mean g) T: the second
    // sum and the template's own sum (for the final mean residual) are
    // formed once here
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c) { gx[r][c] = gx[r][c] - mgx; gy[r][c] = gy[r][c] - mgy; }
    double cTx, cTy, sT;
    {
        double src[2][RB][CB];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < CB; ++c) { src[0][r][c] = gx[r][c]; src[1][r][c] = gy[r][c]; }
        double pa[2][2], pb[1][2];
        rows_partial<L, 2, true>(src, T, pa);
        rows_partial<L, 1, false>(&T, T, pb);
        double p3[3][2], s3[3];
#pragma unroll
        for (int k = 0; k < 2; ++k) { p3[0][k] = pa[0][k]; p3[1][k] = pa[1][k]; p3[2][k] = pb[0][k]; }
        rows_finish<L, 3>(p3, s3);
        cTx = s3[0];
        cTy = s3[1];
        sT = s3[2];
    }

    double ui = 0.0, vi = 0.0;
    if (has_un) {
        ui = 2.0 * ((1.0 - bay) * ((1.0 - bax) * u00 + bax * u01) + bay * ((1.0 - bax) * u10 + bax * u11));
        vi = 2.0 * ((1.0 - bay) * ((1.0 - bax) * v00 + bax * v01) + bay * ((1.0 - bax) * v10 + bax * v11));
    }
    const double a11 = h11 + a.lam, a22 = h22 + a.lam, a12 = h12;
    const double idet = 1.0 / (a11 * a22 - a12 * a12);
    const double m11 = a22 * idet, m12 = -a12 * idet, m22 = a11 * idet;
    const double lim = (double)(W + H + 2 * PS + 4);

    double* win = s_win + (size_t)(threadIdx.x / LPP) * RW::SIZE;
    const auto* __restrict__ J1 = a.J1;
    const int wu = (int)fmin(fmax(floor(ui), -lim), lim), wv = (int)fmin(fmax(floor(vi), -lim), lim);
    rows_window_fill<PS, NRB, NH, R, LPP>(win, J1, W, H, x0 + wu - R, y0 + wv - R, lane);

    constexpr int HALVES = NH == 1 ? 2 : 1, HC = CB / HALVES, GPL = L::GPL, RG = L::RG;
    int wu_ = wu, wv_ = wv;
    // the warped pixels Q = I1(x + u) of the lane, row by row, folded into
    // the canonical partial sums as they are formed: PROD = the two sums of
    // the centred gradients times Q, else the sum of Q
    auto warp_sums = [&](double uu, double vv, auto prod_tag, double (&part)[2][2]) {
        constexpr bool PROD = decltype(prod_tag)::value;
        const double fu = floor(uu), fv = floor(vv);
        const double ax = uu - fu, ay = vv - fv;
        const int iu = (int)fmin(fmax(fu, -lim), lim);
        const int iv = (int)fmin(fmax(fv, -lim), lim);
        if (iu - wu_ < -R || iu - wu_ > R || iv - wv_ < -R || iv - wv_ > R) {
            // left the window: reload it around the current position
            wu_ = iu;
            wv_ = iv;
            rows_window_fill<PS, NRB, NH, R, LPP>(win, J1, W, H, x0 + wu_ - R, y0 + wv_ - R, lane);
        }
        // taps of the lane's rows r0 .. r0 + RB (one more below) and columns
        // c0 .. c0 + CB, interpolated horizontally once per tap row
        const double* base = win + (iv - wv_ + R + r0) * RW::PITCH + (iu - wu_ + R + c0);
        double acc[2][HALVES][GPL];
        double hp[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) hp[c] = fma(ax, base[c + 1] - base[c], base[c]);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const double* row = base + (r + 1) * RW::PITCH;
            double dr[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const double hn = fma(ax, row[c + 1] - row[c], row[c]);
                dr[c] = fma(ay, hn - hp[c], hp[c]);
                hp[c] = hn;
            }
            const int g = r / RG, rr = r - g * RG;
#pragma unroll
            for (int h = 0; h < HALVES; ++h) {
                const int cb = h * HC;
                double s0, s1 = 0.0;
                if constexpr (PROD) {
                    s0 = gx[r][cb] * dr[cb];
                    s1 = gy[r][cb] * dr[cb];
#pragma unroll
                    for (int c = 1; c < HC; ++c) {
                        s0 = fma(gx[r][cb + c], dr[cb + c], s0);
                        s1 = fma(gy[r][cb + c], dr[cb + c], s1);
                    }
                } else {
                    s0 = dr[cb];
#pragma unroll
                    for (int c = 1; c < HC; ++c) s0 = s0 + dr[cb + c];
                }
                acc[0][h][g] = rr == 0 ? s0 : acc[0][h][g] + s0;
                acc[1][h][g] = rr == 0 ? s1 : acc[1][h][g] + s1;
            }
        }
        // binary tree over the lane's row groups
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int h = 0; h < HALVES; ++h) {
#pragma unroll
                for (int step = 1; step < GPL; step <<= 1)
#pragma unroll
                    for (int g = 0; g < GPL; g += 2 * step) acc[m][h][g] = acc[m][h][g] + acc[m][h][g + step];
                part[m][h] = acc[m][h][0];
            }
    };

    double u = ui, v = vi;
    for (int it = 0; it < a.iters; ++it) {
        double part[2][2], s2[2];
        warp_sums(u, v, std::true_type{}, part);
        rows_finish<L, 2>(part, s2);
        const double b1 = s2[0] - cTx, b2 = s2[1] - cTy;
        if (a.stereo) {
            u = u - b1 / a11;   // App. I: one degree of freedom, v stays at its start (zero)
        } else {
            u = u - (m11 * b1 + m12 * b2);
            v = v - (m12 * b1 + m22 * b2);
        }
    }
    // reset test (Sec. 2.2 step 4), then one more warp at the final u for
    // the mean residual
    const double eu = u - ui, ev = v - vi;
    const double moved = sqrt(eu * eu + ev * ev);
    if (moved > (double)PS) { u = ui; v = vi; }
    double md0;
    {
        double part[2][2], s1[1];
        warp_sums(u, v, std::false_type{}, part);
        double p1[1][2] = {{part[0][0], part[0][1]}};
        rows_finish<L, 1>(p1, s1);
        md0 = (s1[0] - sT) / (double)(PS * PS);
    }
    if (valid && lane == 0) {
        auto* P = dis_global(a.patch) + (size_t)pi * 4;
        P[0] = u; P[1] = v; P[2] = md0; P[3] = moved;
        dis_global(a.uinit)[(size_t)pi * 2] = ui;
        dis_global(a.uinit)[(size_t)pi * 2 + 1] = vi;
    }
}
