// Set-up of one refinement tile (Sec. 2.3), shared by the forward tile
// kernel and the reverse (adjoint) tile kernel: the tile geometry, the LDS
// layout, and the per-pixel SOR coefficients of the owned pixels.
#pragma once
#include <hip/hip_runtime.h>
#include "dis_internal.h"

namespace dis_tile {

// U on the region (uu, uv), kept in LDS unless the tile is lean.
template <int N, bool KEEP>
struct RegionU {
    double uu[N], uv[N];
};
template <int N>
struct RegionU<N, false> {};

// LDS of one refinement tile: the core (TW x TH) grows by up to K = DIS_KMAX
// pixels per side (the region); the image tile grows by 2 more for the
// second differences.  The edge-weight planes first hold U + dUf (one more
// row and column, for the forward differences of E_S); the increments share
// storage with the image tile, which is dead by the time they are stored.  A
// lean tile keeps no copy of U on the region (its set-up and store read U
// from memory, where the same values are), so that two 512-thread blocks of
// the larger cores fit one CU.
template <int TW, int TH, int KG = DIS_KMAX, bool LEAN = false>
struct RefineSmem : RegionU<(TH + 2 * KG) * (TW + 2 * KG + 1), !LEAN> {
    static constexpr int K = KG;                     // largest growth of the core on each side
    static constexpr int RWM = TW + 2 * K, RHM = TH + 2 * K;
    static constexpr int LP = RWM + 1;               // region row pitch
    static constexpr int IWM = RWM + 4, IHM = RHM + 4;
    static constexpr int IP = IWM + 1;               // image-tile row pitch
    double wr[(RHM + 1) * LP];                      // U + dUf (u), then the weight of the edge to the right
    double wd[(RHM + 1) * LP];                      // U + dUf (v), then the weight of the edge below
    union {
        struct { double t0[IHM * IP], t1[IHM * IP]; } img;   // J0 / J1w
        struct { double du[RHM * LP], dv[RHM * LP]; } inc;
    } u;
};

// Core, region (core grown by kh on every cut side) and image tile (region
// grown by 2 more) of tile `tile` of a W x H level.
struct TileGeom {
    int W, H;
    int cx0, cy0, cx1, cy1;   // core
    int rx0, ry0, RW, RH;     // region
    int ix0, iy0;             // image tile origin
    int npw;                  // pixel pairs per region row
};

template <int TW, int TH>
__device__ __forceinline__ TileGeom tile_geom(int W, int H, int tiles_x, int tile, int kh) {
    TileGeom g;
    g.W = W;
    g.H = H;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    g.cx0 = tx * TW;
    g.cy0 = ty * TH;
    g.cx1 = min(g.cx0 + TW, W);
    g.cy1 = min(g.cy0 + TH, H);
    g.rx0 = max(g.cx0 - kh, 0);
    g.ry0 = max(g.cy0 - kh, 0);
    const int rx1 = min(g.cx1 + kh, W), ry1 = min(g.cy1 + kh, H);
    g.RW = rx1 - g.rx0;
    g.RH = ry1 - g.ry0;
    g.ix0 = max(g.rx0 - 2, 0);
    g.iy0 = max(g.ry0 - 2, 0);
    g.npw = (g.RW + 1) / 2;
    return g;
}

// SOR coefficients of the owned pixels: PPT pixel pairs per thread, pair
// pr = thread + k NT at region row ly and pair m of that row; the pixel of
// colour c sits at column 2m + ((rx0 + y) & 1) ^ c.
template <int PPT>
struct TileCoef {
    int l[PPT][2];            // region index (row pitch LP), -1 = not owned
    int m[PPT][2];            // neighbours inside the region: 1 right, 2 left, 4 down, 8 up
    double wr[PPT][2], wl[PPT][2], wd[PPT][2], wu[PPT][2];
    double a12[PPT][2], i1[PPT][2], i2[PPT][2], c1[PPT][2], c2[PPT][2];
};

// A lean tile keeps its registers for two blocks per CU: the owned pixels'
// increments and cached linearisation are read where they are used instead
// of being staged in registers with the first loads.
template <int TW, int TH, int NT, int KG = DIS_KMAX, bool LEAN = false>
struct TileShape {
    using S = RefineSmem<TW, TH, KG>;
    static constexpr int PPT = ((S::RWM + 1) / 2 * S::RHM + NT - 1) / NT;
    static constexpr bool kStage = PPT <= 2 && NT <= 512 && !LEAN;   // register budget of 1024-thread blocks
    static constexpr int NS = kStage ? PPT : 1;
    static constexpr bool kLin = PPT <= 2 && NT <= 512;     // linearisation may come from the level's cache
    static constexpr bool kLinPf = kLin && !LEAN;           // ... staged in registers with the first loads
    static constexpr int NL = kLinPf ? PPT : 1;
};

// Steps 1-3 of a tile: one round of global loads (U + dUf on the region plus
// one column / row into wr / wd, U on the region, J0 and the warped J1w on
// the image tile; with few pairs per thread the frozen and starting
// increments of the owned pixels go to registers), the smoothness weights,
// and the coefficients.  Owned pixels farther than `reach` (Chebyshev
// distance) from the core get no coefficients and load no linearisation:
// the caller never updates them (their starting increments and weights are
// still set).  Ends with the image tile still live; the caller places a
// barrier before reusing it.
template <int TW, int TH, int NT, int KG = DIS_KMAX, bool COLOUR = false, bool LEAN = false>
__device__ __forceinline__ void refine_setup(const RefineArgs& a, const TileGeom& g, RefineSmem<TW, TH, KG, LEAN>& sm,
                                             TileCoef<TileShape<TW, TH, NT, KG, LEAN>::PPT>& C,
                                             double (&s_iu)[TileShape<TW, TH, NT, KG, LEAN>::NS][2],
                                             double (&s_iv)[TileShape<TW, TH, NT, KG, LEAN>::NS][2],
                                             int reach = 1 << 20) {
    using S = RefineSmem<TW, TH, KG, LEAN>;
    constexpr int LP = S::LP, IP = S::IP;
    using Shape = TileShape<TW, TH, NT, KG, LEAN>;
    constexpr int PPT = Shape::PPT;
    constexpr bool kStage = Shape::kStage;
    const int W = g.W, H = g.H;
    const size_t n = (size_t)W * H;
    const int rx0 = g.rx0, ry0 = g.ry0, RW = g.RW, RH = g.RH, npw = g.npw;
    const int ix0 = g.ix0, iy0 = g.iy0;
    const auto* __restrict__ U = dis_global(a.U);
    const auto* __restrict__ F = dis_global(a.dUf);
    const auto* __restrict__ Din = dis_global(a.dUin);

    constexpr bool kLin = Shape::kLin;
    constexpr bool kLinPf = Shape::kLinPf;
    constexpr int NL = Shape::NL;
    const bool lin_load = kLin && a.lin_mode == 2;
    constexpr bool colour = COLOUR;   // lin_mode 3: per-channel linearisation
    double s_fu[kStage ? PPT : 1][2], s_fv[kStage ? PPT : 1][2];
    double s_lin[NL][2][11];
    bool far[PPT][2];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pr = threadIdx.x + k * NT;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            C.l[k][c] = -1;
            far[k][c] = true;
            if constexpr (kStage) { s_fu[k][c] = s_fv[k][c] = s_iu[k][c] = s_iv[k][c] = 0.0; }
            if (pr >= npw * RH) continue;
            const int ly = pr / npw, m = pr - ly * npw;
            const int lx = 2 * m + (((rx0 + ry0 + ly) & 1) ^ c);
            if (lx >= RW) continue;
            C.l[k][c] = ly * LP + lx;
            const int x = rx0 + lx, y = ry0 + ly;
            far[k][c] = max(max(max(g.cx0 - x, x - (g.cx1 - 1)), max(g.cy0 - y, y - (g.cy1 - 1))), 0) > reach;
            const size_t gi = (size_t)y * W + x;
            if constexpr (kStage) {
                if (Din) { s_iu[k][c] = Din[gi]; s_iv[k][c] = Din[n + gi]; }
                if (far[k][c]) continue;
                if (F) { s_fu[k][c] = F[gi]; s_fv[k][c] = F[n + gi]; }
            }
            if (far[k][c]) continue;
            if constexpr (kLinPf) {
                if (lin_load) {
#pragma unroll
                    for (int q = 0; q < 11; ++q) s_lin[k][c][q] = dis_global(a.lin)[q * n + gi];
                }
            }
        }
    }

    // 1. loads
    {
        const int ex1 = min(rx0 + RW + 1, W), ey1 = min(ry0 + RH + 1, H);
        const int EW = ex1 - rx0, EH = ey1 - ry0;
#pragma unroll 2
        for (int i = threadIdx.x; i < EW * EH; i += NT) {
            const int ly = i / EW, lx = i - ly * EW;
            const size_t gi = (size_t)(ry0 + ly) * W + rx0 + lx;
            const double u0 = U[gi], v0 = U[n + gi];
            sm.wr[ly * LP + lx] = F ? u0 + F[gi] : u0;
            sm.wd[ly * LP + lx] = F ? v0 + F[n + gi] : v0;
            if constexpr (!LEAN) {
                if (lx < RW && ly < RH) {
                    sm.uu[ly * LP + lx] = u0;
                    sm.uv[ly * LP + lx] = v0;
                }
            }
        }
        const int ix1 = min(rx0 + RW + 2, W), iy1 = min(ry0 + RH + 2, H);
        const int IW = ix1 - ix0, IH = (lin_load || colour) ? 0 : iy1 - iy0;
#pragma unroll 2
        for (int i = threadIdx.x; i < IW * IH; i += NT) {
            const int ly = i / IW, lx = i - ly * IW;
            const size_t gi = (size_t)(iy0 + ly) * W + ix0 + lx;
            sm.u.img.t0[ly * IP + lx] = dis_global(a.J0)[gi];
            sm.u.img.t1[ly * IP + lx] = dis_global(a.J1w)[gi];
        }
    }
    __syncthreads();
    // 2. smoothness weight alpha / (2 sqrt(E_S + eps^2)) of every owned
    //    pixel, from forward differences (zero across the last column / row)
    const double eps2 = a.eps * a.eps;
    double c_ws[PPT][2];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            c_ws[k][c] = 0.0;
            const int e = C.l[k][c];
            if (e < 0) continue;
            const int ly = e / LP, lx = e - ly * LP;
            const int x = rx0 + lx, y = ry0 + ly;
            const double u0 = sm.wr[e], v0 = sm.wd[e];
            double dxu = 0.0, dyu = 0.0, dxv = 0.0, dyv = 0.0;
            if (x < W - 1) { dxu = sm.wr[e + 1] - u0; dxv = sm.wd[e + 1] - v0; }
            if (y < H - 1) { dyu = sm.wr[e + LP] - u0; dyv = sm.wd[e + LP] - v0; }
            const double es = ((dxu * dxu + dyu * dyu) + dxv * dxv) + dyv * dyv;
            c_ws[k][c] = a.alpha / (2.0 * sqrt(es + eps2));
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int e = C.l[k][c];
            if (e < 0) continue;
            const int ly = e / LP, lx = e - ly * LP;
            sm.wr[e] = rx0 + lx < W - 1 ? c_ws[k][c] : 0.0;
            sm.wd[e] = ry0 + ly < H - 1 ? c_ws[k][c] : 0.0;
        }
    }
    __syncthreads();

    // 3. per owned pixel: linearisation (central differences [-1 0 1]/2 with
    //    replicated borders of (J0+J1w)/2 and of J1w - J0, the normalisations
    //    beta), robust data weights at the frozen increment, SOR coefficients
    const double om = a.omega;
    {
        const double* t0 = sm.u.img.t0;
        const double* t1 = sm.u.img.t1;
        // image-tile index of a position already clamped to the image
        auto li = [&](int x, int y) { return (y - iy0) * IP + (x - ix0); };
        auto Ib = [&](int x, int y) { const int l = li(x, y); return 0.5 * (t0[l] + t1[l]); };
        auto Ixa = [&](int x, int y) {
            return (Ib(min(x + 1, W - 1), y) - Ib(max(x - 1, 0), y)) / 2.0;
        };
        auto Iya = [&](int x, int y) {
            return (Ib(x, min(y + 1, H - 1)) - Ib(x, max(y - 1, 0))) / 2.0;
        };
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                C.m[k][c] = 0;
                C.wr[k][c] = C.wl[k][c] = C.wd[k][c] = C.wu[k][c] = 0.0;
                C.a12[k][c] = C.i1[k][c] = C.i2[k][c] = C.c1[k][c] = C.c2[k][c] = 0.0;
                const int l = C.l[k][c];
                if (l < 0 || far[k][c]) continue;
                const int ly = l / LP, lx = l - ly * LP;
                const int x = rx0 + lx, y = ry0 + ly;
                const size_t gi = (size_t)y * W + x;
                double fu, fv;
                if constexpr (kStage) { fu = s_fu[k][c]; fv = s_fv[k][c]; }
                else { fu = F ? F[gi] : 0.0; fv = F ? F[n + gi] : 0.0; }
                double A11, A12, A22, B1, B2;
                if constexpr (colour) {
                    // App. B i: both data energies are channel sums inside one
                    // robust function each; the system sums the channels'
                    // terms at those weights (channel 0 first)
                    double ei = 0.0, eg = 0.0;
                    for (int ch = 0; ch < a.nc; ++ch) {
                        const auto* Lc = dis_global(a.lin) + (size_t)ch * 11 * n + gi;
                        const double cri = (Lc[0] * fu + Lc[n] * fv) + Lc[2 * n];
                        const double crx = (Lc[3 * n] * fu + Lc[4 * n] * fv) + Lc[6 * n];
                        const double cry = (Lc[4 * n] * fu + Lc[5 * n] * fv) + Lc[7 * n];
                        ei = ei + Lc[8 * n] * (cri * cri);
                        eg = eg + (Lc[9 * n] * (crx * crx) + Lc[10 * n] * (cry * cry));
                    }
                    const double pi_ = a.delta / (2.0 * sqrt(ei + eps2));
                    const double pg = a.gamma / (2.0 * sqrt(eg + eps2));
                    A11 = A12 = A22 = B1 = B2 = 0.0;
                    for (int ch = 0; ch < a.nc; ++ch) {
                        const auto* Lc = dis_global(a.lin) + (size_t)ch * 11 * n + gi;
                        const double cIx = Lc[0], cIy = Lc[n], cIz = Lc[2 * n], cIxx = Lc[3 * n], cIxy = Lc[4 * n];
                        const double cIyy = Lc[5 * n], cIxz = Lc[6 * n], cIyz = Lc[7 * n];
                        const double cb0 = Lc[8 * n], cbx = Lc[9 * n], cby = Lc[10 * n];
                        A11 = (A11 + ((pi_ * cb0) * cIx) * cIx) + pg * (((cbx * cIxx) * cIxx) + ((cby * cIxy) * cIxy));
                        A12 = (A12 + ((pi_ * cb0) * cIx) * cIy) + pg * (((cbx * cIxx) * cIxy) + ((cby * cIxy) * cIyy));
                        A22 = (A22 + ((pi_ * cb0) * cIy) * cIy) + pg * (((cbx * cIxy) * cIxy) + ((cby * cIyy) * cIyy));
                        B1 = (B1 + ((pi_ * cb0) * cIx) * cIz) + pg * (((cbx * cIxx) * cIxz) + ((cby * cIxy) * cIyz));
                        B2 = (B2 + ((pi_ * cb0) * cIy) * cIz) + pg * (((cbx * cIxy) * cIxz) + ((cby * cIyy) * cIyz));
                    }
                } else {
                double Ix = 0.0, Iy = 0.0, Iz = 0.0, Ixx = 0.0, Ixy = 0.0, Iyy = 0.0, Ixz = 0.0, Iyz = 0.0;
                double b0 = 0.0, bx = 0.0, by = 0.0;
                bool cached = false;
                if constexpr (kLin) {
                    if (lin_load) {
                        double q[11];
#pragma unroll
                        for (int i = 0; i < 11; ++i) {
                            if constexpr (kLinPf) q[i] = s_lin[k][c][i];
                            else q[i] = dis_global(a.lin)[i * n + gi];
                        }
                        Ix = q[0]; Iy = q[1]; Iz = q[2];
                        Ixx = q[3]; Ixy = q[4]; Iyy = q[5];
                        Ixz = q[6]; Iyz = q[7];
                        b0 = q[8]; bx = q[9]; by = q[10];
                        cached = true;
                    }
                }
                if (!cached) {
                    const int xm = max(x - 1, 0), xp = min(x + 1, W - 1);
                    const int ym = max(y - 1, 0), yp = min(y + 1, H - 1);
                    Ix = Ixa(x, y);
                    Iy = Iya(x, y);
                    const int lc = li(x, y);
                    Iz = t1[lc] - t0[lc];
                    Ixx = (Ixa(xp, y) - Ixa(xm, y)) / 2.0;
                    Ixy = (Ixa(x, yp) - Ixa(x, ym)) / 2.0;
                    Iyy = (Iya(x, yp) - Iya(x, ym)) / 2.0;
                    const int lxp = li(xp, y), lxm = li(xm, y), lyp = li(x, yp), lym = li(x, ym);
                    Ixz = (t1[lxp] - t1[lxm]) / 2.0 - (t0[lxp] - t0[lxm]) / 2.0;
                    Iyz = (t1[lyp] - t1[lym]) / 2.0 - (t0[lyp] - t0[lym]) / 2.0;
                    b0 = 1.0 / ((Ix * Ix + Iy * Iy) + 0.01);
                    bx = 1.0 / ((Ixx * Ixx + Ixy * Ixy) + 0.01);
                    by = 1.0 / ((Ixy * Ixy + Iyy * Iyy) + 0.01);
                    if (a.lin_mode == 1 && x >= g.cx0 && x < g.cx1 && y >= g.cy0 && y < g.cy1) {
                        auto* Lo = dis_global(a.lin) + gi;
                        Lo[0] = Ix; Lo[n] = Iy; Lo[2 * n] = Iz; Lo[3 * n] = Ixx; Lo[4 * n] = Ixy;
                        Lo[5 * n] = Iyy; Lo[6 * n] = Ixz; Lo[7 * n] = Iyz; Lo[8 * n] = b0; Lo[9 * n] = bx;
                        Lo[10 * n] = by;
                    }
                }
                const double ri = (Ix * fu + Iy * fv) + Iz;
                const double ei = b0 * (ri * ri);
                const double rx = (Ixx * fu + Ixy * fv) + Ixz;
                const double ry = (Ixy * fu + Iyy * fv) + Iyz;
                const double eg = bx * (rx * rx) + by * (ry * ry);
                const double pi_ = a.delta / (2.0 * sqrt(ei + eps2));
                const double pg = a.gamma / (2.0 * sqrt(eg + eps2));
                A11 = ((pi_ * b0) * Ix) * Ix + pg * (((bx * Ixx) * Ixx) + ((by * Ixy) * Ixy));
                A12 = ((pi_ * b0) * Ix) * Iy + pg * (((bx * Ixx) * Ixy) + ((by * Ixy) * Iyy));
                A22 = ((pi_ * b0) * Iy) * Iy + pg * (((bx * Ixy) * Ixy) + ((by * Iyy) * Iyy));
                B1 = ((pi_ * b0) * Ix) * Iz + pg * (((bx * Ixx) * Ixz) + ((by * Ixy) * Iyz));
                B2 = ((pi_ * b0) * Iy) * Iz + pg * (((bx * Ixy) * Ixz) + ((by * Iyy) * Iyz));
                }
                // edges: right/down owned by this pixel, left/up by the
                // neighbour; neighbours outside the region (not the image) are
                // dropped, which only disturbs pixels the erosion discards
                const bool hr = x < W - 1 && lx + 1 < RW, hl = x > 0 && lx > 0;
                const bool hd = y < H - 1 && ly + 1 < RH, hu = y > 0 && ly > 0;
                const double wr = hr ? sm.wr[l] : 0.0, wl = hl ? sm.wr[l - 1] : 0.0;
                const double wd = hd ? sm.wd[l] : 0.0, wu = hu ? sm.wd[l - LP] : 0.0;
                const double Ssum = ((wr + wl) + wd) + wu;
                double Up, Vp, Ur, Ul, Ud, Uu, Vr, Vl, Vd, Vu;
                if constexpr (LEAN) {
                    // the same values, from memory (gi: the pixel; its neighbours one column / row away)
                    Up = U[gi]; Vp = U[n + gi];
                    Ur = hr ? U[gi + 1] : 0.0; Ul = hl ? U[gi - 1] : 0.0;
                    Ud = hd ? U[gi + W] : 0.0; Uu = hu ? U[gi - W] : 0.0;
                    Vr = hr ? U[n + gi + 1] : 0.0; Vl = hl ? U[n + gi - 1] : 0.0;
                    Vd = hd ? U[n + gi + W] : 0.0; Vu = hu ? U[n + gi - W] : 0.0;
                } else {
                    Up = sm.uu[l]; Vp = sm.uv[l];
                    Ur = hr ? sm.uu[l + 1] : 0.0; Ul = hl ? sm.uu[l - 1] : 0.0;
                    Ud = hd ? sm.uu[l + LP] : 0.0; Uu = hu ? sm.uu[l - LP] : 0.0;
                    Vr = hr ? sm.uv[l + 1] : 0.0; Vl = hl ? sm.uv[l - 1] : 0.0;
                    Vd = hd ? sm.uv[l + LP] : 0.0; Vu = hu ? sm.uv[l - LP] : 0.0;
                }
                const double NU = ((wr * Ur + wl * Ul) + wd * Ud) + wu * Uu;
                const double NV = ((wr * Vr + wl * Vl) + wd * Vd) + wu * Vu;
                C.m[k][c] = (hr ? 1 : 0) | (hl ? 2 : 0) | (hd ? 4 : 0) | (hu ? 8 : 0);
                C.wr[k][c] = wr; C.wl[k][c] = wl; C.wd[k][c] = wd; C.wu[k][c] = wu;
                C.a12[k][c] = A12;
                C.i1[k][c] = om / (A11 + Ssum);
                C.i2[k][c] = om / (A22 + Ssum);
                C.c1[k][c] = (NU - Ssum * Up) - B1;
                C.c2[k][c] = (NV - Ssum * Vp) - B2;
            }
        }
    }
}

}  // namespace dis_tile
