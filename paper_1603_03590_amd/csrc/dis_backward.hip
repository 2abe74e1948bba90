// Adjoint (reverse-mode) kernels of Dense Inverse Search for gfx950.
//
// The forward pipeline (Alg. 1 with the readings of the forward kernels) is
// differentiated step by step: upscaling, the refinement's fixed-point steps
// (red-black SOR sweeps replayed in reverse from a tape of their states, then
// the frozen robust weights and the linearisation), the warped second frame,
// the densification of Eq. (3), the unrolled inverse-compositional
// Gauss-Newton iterations with the reset test, the patch initialisation from
// the coarser flow, and the box pyramid.  float64 throughout; contributions
// that several threads add to one element use hardware float64 atomics, so
// gradients can differ between runs in the last bits.
#include <hip/hip_runtime.h>

#include <type_traits>
#include "dis_backward.h"
#include "dis_refine_tile.h"
#include "dis_lanes.h"

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ void atom(double* p, double v) {
    if (v != 0.0) unsafeAtomicAdd(p, v);
}

// Bilinear taps of (x, y) in a W x H image (pixel values at integer
// coordinates, indices clamped), their weights, and the value's partial
// derivatives with respect to x and y.
struct Taps {
    int i00, i01, i10, i11;
    int fx, fy;             // floor of the position before any clamp
    double w00, w01, w10, w11;
    double val, dx, dy;
};

__device__ __forceinline__ Taps taps_of(const double* img, int W, int H, double x, double y) {
    double xf = floor(x), yf = floor(y);
    const double ax = x - xf, ay = y - yf;
    Taps t;
    t.fx = (int)xf;
    t.fy = (int)yf;
    xf = fmin(fmax(xf, -2.0), (double)W + 1.0);
    yf = fmin(fmax(yf, -2.0), (double)H + 1.0);
    const int xi = (int)xf, yi = (int)yf;
    const int x0 = clampi(xi, 0, W - 1), x1 = clampi(xi + 1, 0, W - 1);
    const int y0 = clampi(yi, 0, H - 1), y1 = clampi(yi + 1, 0, H - 1);
    t.i00 = y0 * W + x0; t.i01 = y0 * W + x1; t.i10 = y1 * W + x0; t.i11 = y1 * W + x1;
    t.w00 = (1.0 - ay) * (1.0 - ax); t.w01 = (1.0 - ay) * ax; t.w10 = ay * (1.0 - ax); t.w11 = ay * ax;
    const double a = img ? img[t.i00] : 0.0, b = img ? img[t.i01] : 0.0;
    const double c = img ? img[t.i10] : 0.0, d = img ? img[t.i11] : 0.0;
    const double top = (1.0 - ax) * a + ax * b, bot = (1.0 - ax) * c + ax * d;
    t.val = (1.0 - ay) * top + ay * bot;
    t.dx = (1.0 - ay) * (b - a) + ay * (d - c);
    t.dy = bot - top;
    return t;
}

__device__ __forceinline__ void scatter_taps(double* g, const Taps& t, double v) {
    atom(g + t.i00, v * t.w00);
    atom(g + t.i01, v * t.w01);
    atom(g + t.i10, v * t.w10);
    atom(g + t.i11, v * t.w11);
}

// An LDS pointer the compiler knows to be one (a pointer into dynamic shared
// memory that meets a global one in a branch is otherwise accessed through
// flat instructions on both sides).
template <typename T>
__device__ __forceinline__ __attribute__((address_space(3))) T* dis_lds(T* p) {
    return (__attribute__((address_space(3))) T*)p;
}

}  // namespace

// --------------------------------------------------------------- utilities

__global__ __launch_bounds__(256) void k_bzero(const BZeroArgs a) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < a.n) a.p[i] = 0.0;
}

__global__ __launch_bounds__(256) void k_bzero_list(const BZeroList L) {
    int e = 0;
    while (e + 1 < L.cnt && (int)blockIdx.x >= L.start[e + 1]) ++e;
    const size_t i = (size_t)(blockIdx.x - L.start[e]) * 256 + threadIdx.x;
    if (i < L.n[e]) L.p[e][i] = 0.0;
}

// dst = src (and dst2 = src when given)
__global__ __launch_bounds__(256) void k_bcopy(const BCopyArgs a) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    a.dst[i] = a.src[i];
    if (a.dst2) a.dst2[i] = a.src[i];
}

// dst += src
__global__ __launch_bounds__(256) void k_baxpy(const BCopyArgs a) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < a.n) a.dst[i] = a.dst[i] + a.src[i];
}

// --------------------------------------------------------------- upscaling

// flow(x) = f * bilinear(U, x / f): every output pixel hands f * gF to the
// four taps it read.
__global__ __launch_bounds__(256) void k_bwd_upsample(const UpsBwdArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.W || y >= a.H) return;
    double qx, qy;
    if (a.centre_map) { qx = ((double)x + 0.5) / a.f - 0.5; qy = ((double)y + 0.5) / a.f - 0.5; }
    else { qx = (double)x / a.f; qy = (double)y / a.f; }
    const size_t g = (size_t)y * a.W + x, n = (size_t)a.W * a.H;
    const double gu = a.g_f64 ? ((const double*)a.gF)[g] : (double)((const float*)a.gF)[g];
    const double gv = a.g_f64 ? ((const double*)a.gF)[n + g] : (double)((const float*)a.gF)[n + g];
    const Taps t = taps_of(nullptr, a.Ws, a.Hs, qx, qy);
    const size_t ns = (size_t)a.Ws * a.Hs;
    scatter_taps(a.gU, t, a.f * gu);
    scatter_taps(a.gU + ns, t, a.f * gv);
}

// ------------------------------------------------------------- refinement

namespace {

// Linearisation and SOR coefficients of pixel (x, y) at the frozen increment
// F (same formulas and order as the forward refinement tile).
struct Lin {
    double Ix, Iy, Iz, Ixx, Ixy, Iyy, Ixz, Iyz, b0, bx, by;
    double fu, fv, ri, rx, ry, ei, eg, pi, pg;
    double A11, A12, A22, B1, B2;
};

__device__ __forceinline__ Lin lin_at(const RefBwdArgs& a, int x, int y) {
    const int W = a.W, H = a.H;
    const double* A = a.J0;
    const double* B = a.J1w;
    auto Ib = [&](int xx, int yy) { return 0.5 * (A[yy * W + xx] + B[yy * W + xx]); };
    auto Ixa = [&](int xx, int yy) { return (Ib(min(xx + 1, W - 1), yy) - Ib(max(xx - 1, 0), yy)) / 2.0; };
    auto Iya = [&](int xx, int yy) { return (Ib(xx, min(yy + 1, H - 1)) - Ib(xx, max(yy - 1, 0))) / 2.0; };
    const int xm = max(x - 1, 0), xp = min(x + 1, W - 1), ym = max(y - 1, 0), yp = min(y + 1, H - 1);
    const size_t g = (size_t)y * W + x, n = (size_t)W * H;
    Lin L;
    L.Ix = Ixa(x, y);
    L.Iy = Iya(x, y);
    L.Iz = B[g] - A[g];
    L.Ixx = (Ixa(xp, y) - Ixa(xm, y)) / 2.0;
    L.Ixy = (Ixa(x, yp) - Ixa(x, ym)) / 2.0;
    L.Iyy = (Iya(x, yp) - Iya(x, ym)) / 2.0;
    L.Ixz = (B[y * W + xp] - B[y * W + xm]) / 2.0 - (A[y * W + xp] - A[y * W + xm]) / 2.0;
    L.Iyz = (B[yp * W + x] - B[ym * W + x]) / 2.0 - (A[yp * W + x] - A[ym * W + x]) / 2.0;
    L.b0 = 1.0 / ((L.Ix * L.Ix + L.Iy * L.Iy) + 0.01);
    L.bx = 1.0 / ((L.Ixx * L.Ixx + L.Ixy * L.Ixy) + 0.01);
    L.by = 1.0 / ((L.Ixy * L.Ixy + L.Iyy * L.Iyy) + 0.01);
    L.fu = a.F ? a.F[g] : 0.0;
    L.fv = a.F ? a.F[n + g] : 0.0;
    const double eps2 = a.eps * a.eps;
    L.ri = (L.Ix * L.fu + L.Iy * L.fv) + L.Iz;
    L.ei = L.b0 * (L.ri * L.ri);
    L.rx = (L.Ixx * L.fu + L.Ixy * L.fv) + L.Ixz;
    L.ry = (L.Ixy * L.fu + L.Iyy * L.fv) + L.Iyz;
    L.eg = L.bx * (L.rx * L.rx) + L.by * (L.ry * L.ry);
    L.pi = a.delta / (2.0 * sqrt(L.ei + eps2));
    L.pg = a.gamma / (2.0 * sqrt(L.eg + eps2));
    const double pi = L.pi, pg = L.pg;
    L.A11 = ((pi * L.b0) * L.Ix) * L.Ix + pg * (((L.bx * L.Ixx) * L.Ixx) + ((L.by * L.Ixy) * L.Ixy));
    L.A12 = ((pi * L.b0) * L.Ix) * L.Iy + pg * (((L.bx * L.Ixx) * L.Ixy) + ((L.by * L.Ixy) * L.Iyy));
    L.A22 = ((pi * L.b0) * L.Iy) * L.Iy + pg * (((L.bx * L.Ixy) * L.Ixy) + ((L.by * L.Iyy) * L.Iyy));
    L.B1 = ((pi * L.b0) * L.Ix) * L.Iz + pg * (((L.bx * L.Ixx) * L.Ixz) + ((L.by * L.Ixy) * L.Iyz));
    L.B2 = ((pi * L.b0) * L.Iy) * L.Iz + pg * (((L.bx * L.Ixy) * L.Ixz) + ((L.by * L.Iyy) * L.Iyz));
    return L;
}

// Smoothness weight owned by (x, y) from the full flow U + F.
__device__ __forceinline__ double ws_at(const RefBwdArgs& a, int x, int y, double* E = nullptr) {
    const int W = a.W, H = a.H;
    const size_t g = (size_t)y * W + x, n = (size_t)W * H;
    auto uu = [&](size_t i) { return a.F ? a.U[i] + a.F[i] : a.U[i]; };
    auto vv = [&](size_t i) { return a.F ? a.U[n + i] + a.F[n + i] : a.U[n + i]; };
    const double u0 = uu(g), v0 = vv(g);
    double dxu = 0.0, dyu = 0.0, dxv = 0.0, dyv = 0.0;
    if (x < W - 1) { dxu = uu(g + 1) - u0; dxv = vv(g + 1) - v0; }
    if (y < H - 1) { dyu = uu(g + W) - u0; dyv = vv(g + W) - v0; }
    const double es = ((dxu * dxu + dyu * dyu) + dxv * dxv) + dyv * dyv;
    if (E) *E = es;
    return a.alpha / (2.0 * sqrt(es + a.eps * a.eps));
}

}  // namespace

// Coefficients of one fixed-point step, per pixel: A12, omega/(A11+S),
// omega/(A22+S), c1, c2 (the constant parts of the SOR updates) and the edge
// weight ws the pixel owns (right and lower edge).
__global__ __launch_bounds__(256) void k_bwd_coef(const RefBwdArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int W = a.W, H = a.H;
    if (x >= W || y >= H) return;
    const size_t g = (size_t)y * W + x, n = (size_t)W * H;
    a.coef[5 * n + g] = ws_at(a, x, y);
}

__global__ __launch_bounds__(256) void k_bwd_coef2(const RefBwdArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int W = a.W, H = a.H;
    if (x >= W || y >= H) return;
    const size_t g = (size_t)y * W + x, n = (size_t)W * H;
    const double* ws = a.coef + 5 * n;
    const Lin L = lin_at(a, x, y);
    const double wr = x < W - 1 ? ws[g] : 0.0, wl = x > 0 ? ws[g - 1] : 0.0;
    const double wd = y < H - 1 ? ws[g] : 0.0, wu = y > 0 ? ws[g - W] : 0.0;
    const double S = ((wr + wl) + wd) + wu;
    const double* U = a.U;
    const double Ur = x < W - 1 ? U[g + 1] : 0.0, Ul = x > 0 ? U[g - 1] : 0.0;
    const double Ud = y < H - 1 ? U[g + W] : 0.0, Uu = y > 0 ? U[g - W] : 0.0;
    const double Vr = x < W - 1 ? U[n + g + 1] : 0.0, Vl = x > 0 ? U[n + g - 1] : 0.0;
    const double Vd = y < H - 1 ? U[n + g + W] : 0.0, Vu = y > 0 ? U[n + g - W] : 0.0;
    const double NU = ((wr * Ur + wl * Ul) + wd * Ud) + wu * Uu;
    const double NV = ((wr * Vr + wl * Vl) + wd * Vd) + wu * Vu;
    a.coef[0 * n + g] = L.A12;
    a.coef[1 * n + g] = a.omega / (L.A11 + S);
    a.coef[2 * n + g] = a.omega / (L.A22 + S);
    a.coef[3 * n + g] = (NU - S * U[g]) - L.B1;
    a.coef[4 * n + g] = (NV - S * U[n + g]) - L.B2;
}

// Reverse of one red-black half sweep, part 1: the pixels of colour c
// (updated by that half sweep).  gd holds the adjoint of the state after the
// half sweep; on exit it holds the adjoint of the state before it for these
// pixels, gn the adjoints of their neighbour sums, and acc the adjoints of
// their coefficients (summed over the step's half sweeps).
__global__ __launch_bounds__(256) void k_bwd_sweep_a(const SweepBwdArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int W = a.W, H = a.H;
    if (x >= W || y >= H || ((x + y) & 1) != a.colour) return;
    const size_t g = (size_t)y * W + x, n = (size_t)W * H;
    const double* ws = a.coef + 5 * n;
    const double* st = a.state;        // state before the half sweep, null = zero
    auto du = [&](size_t i) { return st ? st[i] : 0.0; };
    auto dv = [&](size_t i) { return st ? st[n + i] : 0.0; };
    const bool hr = x < W - 1, hl = x > 0, hd = y < H - 1, hu = y > 0;
    const double wr = hr ? ws[g] : 0.0, wl = hl ? ws[g - 1] : 0.0;
    const double wd = hd ? ws[g] : 0.0, wu = hu ? ws[g - W] : 0.0;
    const double A12 = a.coef[g], i1 = a.coef[n + g], i2 = a.coef[2 * n + g];
    const double c1 = a.coef[3 * n + g], c2 = a.coef[4 * n + g];
    const double om1 = 1.0 - a.omega;
    const double dur = hr ? du(g + 1) : 0.0, dul = hl ? du(g - 1) : 0.0;
    const double dud = hd ? du(g + W) : 0.0, duu = hu ? du(g - W) : 0.0;
    const double dvr = hr ? dv(g + 1) : 0.0, dvl = hl ? dv(g - 1) : 0.0;
    const double dvd = hd ? dv(g + W) : 0.0, dvu = hu ? dv(g - W) : 0.0;
    const double dup = du(g), dvp = dv(g);
    // forward replay of this pixel's update
    const double nu = ((wr * dur + wl * dul) + wd * dud) + wu * duu;
    const double r1 = (nu + c1) - A12 * dvp;
    const double dun = om1 * dup + i1 * r1;
    const double nv = ((wr * dvr + wl * dvl) + wd * dvd) + wu * dvu;
    const double r2 = (nv + c2) - A12 * dun;
    // adjoint
    const double adv = a.gd[n + g];
    const double gr2 = i2 * adv;
    const double adu = a.gd[g] - A12 * gr2;
    const double gr1 = i1 * adu;
    double* acc = a.acc;
    acc[0 * n + g] += r1 * adu;                    // omega/(A11+S)
    acc[1 * n + g] += r2 * adv;                    // omega/(A22+S)
    acc[2 * n + g] += gr1;                         // c1
    acc[3 * n + g] += gr2;                         // c2
    acc[4 * n + g] += -dun * gr2 - dvp * gr1;      // A12
    acc[5 * n + g] += dur * gr1 + dvr * gr2;       // edge weights seen from this pixel: right
    acc[6 * n + g] += dul * gr1 + dvl * gr2;       // left
    acc[7 * n + g] += dud * gr1 + dvd * gr2;       // down
    acc[8 * n + g] += duu * gr1 + dvu * gr2;       // up
    a.gd[g] = om1 * adu;
    a.gd[n + g] = om1 * adv - A12 * gr1;
    a.gn[g] = gr1;
    a.gn[n + g] = gr2;
}

// Part 2: the pixels of the other colour collect what their neighbours'
// updates owe them.
__global__ __launch_bounds__(256) void k_bwd_sweep_b(const SweepBwdArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int W = a.W, H = a.H;
    if (x >= W || y >= H || ((x + y) & 1) == a.colour) return;
    const size_t g = (size_t)y * W + x, n = (size_t)W * H;
    const double* ws = a.coef + 5 * n;
    const bool hr = x < W - 1, hl = x > 0, hd = y < H - 1, hu = y > 0;
    const double wr = hr ? ws[g] : 0.0, wl = hl ? ws[g - 1] : 0.0;
    const double wd = hd ? ws[g] : 0.0, wu = hu ? ws[g - W] : 0.0;
    double su = 0.0, sv = 0.0;
    if (hr) { su += wr * a.gn[g + 1]; sv += wr * a.gn[n + g + 1]; }
    if (hl) { su += wl * a.gn[g - 1]; sv += wl * a.gn[n + g - 1]; }
    if (hd) { su += wd * a.gn[g + W]; sv += wd * a.gn[n + g + W]; }
    if (hu) { su += wu * a.gn[g - W]; sv += wu * a.gn[n + g - W]; }
    a.gd[g] += su;
    a.gd[n + g] += sv;
}

// Adjoints of A11 and A22 (through i = omega / (A + S)), of the pixel's
// weight sum S and of c1, c2 (c = N - S U - B) from the step's coefficient
// adjoints.
struct PixAdj {
    double gA11, gA22, gS, gc1, gc2;
};
__device__ __forceinline__ PixAdj pix_adj(const RefBwdArgs& a, size_t g, size_t n) {
    const double* acc = a.acc;
    const double i1 = a.coef[n + g], i2 = a.coef[2 * n + g];
    const double gi1 = acc[g], gi2 = acc[n + g];
    PixAdj r;
    r.gc1 = acc[2 * n + g];
    r.gc2 = acc[3 * n + g];
    r.gA11 = -gi1 * i1 * i1 / a.omega;
    r.gA22 = -gi2 * i2 * i2 / a.omega;
    r.gS = r.gA11 + r.gA22 - a.U[g] * r.gc1 - a.U[n + g] * r.gc2;
    return r;
}

// The coefficient adjoints of one fixed-point step, part 1 (per pixel):
// through omega/(A+S), c = N - S U - B, the neighbour sums N and S, the
// robust data weights and the linearisation, down to U, F, J0 and J1w.
__device__ __forceinline__ void bwd_lin_pixel(const RefBwdArgs& a, int x, int y, double (&simg)[2][8][68],
                                              double (&sfl)[2][2][6][66], int x0, int y0) {
    const int ox = x0 - 2, oy = y0 - 2;
    // flow adjoints (field 0: U, 1: F; plane c) into the block's LDS cells
    auto fl = [&](int f, int c, int xx, int yy, double v) {
        if (v != 0.0) unsafeAtomicAdd(&sfl[f][c][yy - y0 + 1][xx - x0 + 1], v);
    };
    const int W = a.W, H = a.H;
    const size_t g = (size_t)y * W + x, n = (size_t)W * H;
    const double* ws = a.coef + 5 * n;
    const double* acc = a.acc;
    const bool hr = x < W - 1, hl = x > 0, hd = y < H - 1, hu = y > 0;
    const double wr = hr ? ws[g] : 0.0, wl = hl ? ws[g - 1] : 0.0;
    const double wd = hd ? ws[g] : 0.0, wu = hu ? ws[g - W] : 0.0;
    const double S = ((wr + wl) + wd) + wu;
    const PixAdj pa = pix_adj(a, g, n);
    const double gA11 = pa.gA11, gA22 = pa.gA22, gc1 = pa.gc1, gc2 = pa.gc2;
    const double gA12 = acc[4 * n + g];
    const double gB1 = -gc1, gB2 = -gc2;
    // c = N - S U - B: U at the pixel and its neighbours
    fl(0, 0, x, y, -S * gc1);
    fl(0, 1, x, y, -S * gc2);
    if (hr) { fl(0, 0, x + 1, y, wr * gc1); fl(0, 1, x + 1, y, wr * gc2); }
    if (hl) { fl(0, 0, x - 1, y, wl * gc1); fl(0, 1, x - 1, y, wl * gc2); }
    if (hd) { fl(0, 0, x, y + 1, wd * gc1); fl(0, 1, x, y + 1, wd * gc2); }
    if (hu) { fl(0, 0, x, y - 1, wu * gc1); fl(0, 1, x, y - 1, wu * gc2); }

    // robust data weights and linearisation
    const Lin L = lin_at(a, x, y);
    const double b0 = L.b0, bx = L.bx, by = L.by;
    const double Ix = L.Ix, Iy = L.Iy, Iz = L.Iz, Ixx = L.Ixx, Ixy = L.Ixy, Iyy = L.Iyy, Ixz = L.Ixz, Iyz = L.Iyz;
    const double pi = L.pi, pg = L.pg;
    const double gpi = gA11 * (b0 * Ix * Ix) + gA12 * (b0 * Ix * Iy) + gA22 * (b0 * Iy * Iy) + gB1 * (b0 * Ix * Iz) +
                       gB2 * (b0 * Iy * Iz);
    const double gpg = gA11 * (bx * Ixx * Ixx + by * Ixy * Ixy) + gA12 * (bx * Ixx * Ixy + by * Ixy * Iyy) +
                       gA22 * (bx * Ixy * Ixy + by * Iyy * Iyy) + gB1 * (bx * Ixx * Ixz + by * Ixy * Iyz) +
                       gB2 * (bx * Ixy * Ixz + by * Iyy * Iyz);
    double gb0 = pi * (gA11 * Ix * Ix + gA12 * Ix * Iy + gA22 * Iy * Iy + gB1 * Ix * Iz + gB2 * Iy * Iz);
    double gIx = pi * b0 * (2.0 * gA11 * Ix + gA12 * Iy + gB1 * Iz);
    double gIy = pi * b0 * (gA12 * Ix + 2.0 * gA22 * Iy + gB2 * Iz);
    double gIz = pi * b0 * (gB1 * Ix + gB2 * Iy);
    double gbx = pg * (gA11 * Ixx * Ixx + gA12 * Ixx * Ixy + gA22 * Ixy * Ixy + gB1 * Ixx * Ixz + gB2 * Ixy * Ixz);
    double gby = pg * (gA11 * Ixy * Ixy + gA12 * Ixy * Iyy + gA22 * Iyy * Iyy + gB1 * Ixy * Iyz + gB2 * Iyy * Iyz);
    double gIxx = pg * bx * (2.0 * gA11 * Ixx + gA12 * Ixy + gB1 * Ixz);
    double gIxy = pg * (bx * (gA12 * Ixx + 2.0 * gA22 * Ixy + gB2 * Ixz) + by * (2.0 * gA11 * Ixy + gA12 * Iyy + gB1 * Iyz));
    double gIyy = pg * by * (gA12 * Ixy + 2.0 * gA22 * Iyy + gB2 * Iyz);
    double gIxz = pg * bx * (gB1 * Ixx + gB2 * Ixy);
    double gIyz = pg * by * (gB1 * Ixy + gB2 * Iyy);
    const double eps2 = a.eps * a.eps;
    // psi = w / (2 sqrt(E + eps^2))
    const double gei = -gpi * pi / (2.0 * (L.ei + eps2));
    const double geg = -gpg * pg / (2.0 * (L.eg + eps2));
    gb0 += gei * L.ri * L.ri;
    const double gri = 2.0 * b0 * L.ri * gei;
    gIx += gri * L.fu; gIy += gri * L.fv; gIz += gri;
    double gfu = gri * Ix, gfv = gri * Iy;
    gbx += geg * L.rx * L.rx;
    gby += geg * L.ry * L.ry;
    const double grx = 2.0 * bx * L.rx * geg, gry = 2.0 * by * L.ry * geg;
    gIxx += grx * L.fu; gIxy += grx * L.fv + gry * L.fu; gIxz += grx;
    gIyy += gry * L.fv; gIyz += gry;
    gfu += grx * Ixx + gry * Ixy;
    gfv += grx * Ixy + gry * Iyy;
    if (a.F) { fl(1, 0, x, y, gfu); fl(1, 1, x, y, gfv); }
    // beta = 1 / (a^2 + b^2 + 0.01)
    gIx += gb0 * (-b0 * b0) * 2.0 * Ix; gIy += gb0 * (-b0 * b0) * 2.0 * Iy;
    gIxx += gbx * (-bx * bx) * 2.0 * Ixx; gIxy += gbx * (-bx * bx) * 2.0 * Ixy;
    gIxy += gby * (-by * by) * 2.0 * Ixy; gIyy += gby * (-by * by) * 2.0 * Iyy;
    // derivatives -> images (central differences with replicated borders)
    const int xm = max(x - 1, 0), xp = min(x + 1, W - 1), ym = max(y - 1, 0), yp = min(y + 1, H - 1);
    // image adjoints into the block's LDS cells (J0: 0, J1w: 1)
    auto lds = [&](int f, int xx, int yy, double v) {
        if (v != 0.0) unsafeAtomicAdd(&simg[f][yy - oy][xx - ox], v);
    };
    auto addIb = [&](int xx, int yy, double v) {   // Ib = (J0 + J1w)/2
        lds(0, xx, yy, 0.5 * v);
        lds(1, xx, yy, 0.5 * v);
    };
    auto addIxa = [&](int xx, int yy, double v) {  // Ix at (xx, yy)
        addIb(min(xx + 1, W - 1), yy, v / 2.0);
        addIb(max(xx - 1, 0), yy, -v / 2.0);
    };
    auto addIya = [&](int xx, int yy, double v) {
        addIb(xx, min(yy + 1, H - 1), v / 2.0);
        addIb(xx, max(yy - 1, 0), -v / 2.0);
    };
    addIxa(x, y, gIx);
    addIya(x, y, gIy);
    addIxa(xp, y, gIxx / 2.0);
    addIxa(xm, y, -gIxx / 2.0);
    addIxa(x, yp, gIxy / 2.0);
    addIxa(x, ym, -gIxy / 2.0);
    addIya(x, yp, gIyy / 2.0);
    addIya(x, ym, -gIyy / 2.0);
    lds(1, x, y, gIz);
    lds(0, x, y, -gIz);
    lds(1, xp, y, gIxz / 2.0); lds(1, xm, y, -gIxz / 2.0);
    lds(0, xp, y, -gIxz / 2.0); lds(0, xm, y, gIxz / 2.0);
    lds(1, x, yp, gIyz / 2.0); lds(1, x, ym, -gIyz / 2.0);
    lds(0, x, yp, -gIyz / 2.0); lds(0, x, ym, gIyz / 2.0);
}

// One fixed-point step's coefficient adjoints on a 64x4 block.  Part 1 per
// pixel (bwd_lin_pixel).  Part 2 per owner pixel: the adjoint of the edge
// weights it owns (right and lower edge, each seen from both endpoints: the
// coefficient adjoint of the edge plus the endpoint's dS and dc terms), then
// through ws = alpha / (2 sqrt(E_S + eps^2)) and the forward differences of
// U + F.  The endpoint terms of the block's pixels and of the column to its
// right and the row below it are formed once, into LDS.  Every adjoint the
// block produces lands within 2 pixels of it (the images') or 1 (the flow's
// U and F): they are summed in LDS first (68x8 and 66x6 cells per plane),
// then added to memory once per cell, which takes most of the float64
// atomics off the memory side.
__global__ __launch_bounds__(256) void k_bwd_lin_ws(const RefBwdArgs a) {
    __shared__ double simg[2][8][68];
    __shared__ double sfl[2][2][6][66];
    __shared__ double sadj[3][5][65];   // dS, dc1, dc2
    for (int i = threadIdx.x; i < 2 * 8 * 68; i += 256) (&simg[0][0][0])[i] = 0.0;
    for (int i = threadIdx.x; i < 2 * 2 * 6 * 66; i += 256) (&sfl[0][0][0][0])[i] = 0.0;
    const int W = a.W, H = a.H;
    const size_t n = (size_t)W * H;
    const int x0 = (int)blockIdx.x * 64, y0 = (int)blockIdx.y * 4;
    for (int i = threadIdx.x; i < 5 * 65; i += 256) {
        const int ly = i / 65, lx = i - ly * 65;
        const int xx = x0 + lx, yy = y0 + ly;
        if (xx >= W || yy >= H) continue;
        const PixAdj pa = pix_adj(a, (size_t)yy * W + xx, n);
        sadj[0][ly][lx] = pa.gS;
        sadj[1][ly][lx] = pa.gc1;
        sadj[2][ly][lx] = pa.gc2;
    }
    __syncthreads();
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int x = x0 + lx, y = y0 + ly;
    if (x < W && y < H) {
        bwd_lin_pixel(a, x, y, simg, sfl, x0, y0);
        const size_t g = (size_t)y * W + x;
        const double* acc = a.acc;
        const double* U = a.U;
        // an edge's adjoint as seen from its endpoint ge (block cell cx, cy),
        // whose coefficient adjoint of that edge is plane q; go: the other endpoint
        auto seen = [&](int q, size_t ge, int cx, int cy, size_t go) {
            return ((acc[q * n + ge] + sadj[0][cy][cx]) + sadj[1][cy][cx] * U[go]) + sadj[2][cy][cx] * U[n + go];
        };
        double gws = 0.0;
        if (x < W - 1) gws += seen(5, g, lx, ly, g + 1) + seen(6, g + 1, lx + 1, ly, g);
        if (y < H - 1) gws += seen(7, g, lx, ly, g + W) + seen(8, g + W, lx, ly + 1, g);
        if (gws != 0.0) {
            double es;
            const double ws = ws_at(a, x, y, &es);
            const double gE = -gws * ws / (2.0 * (es + a.eps * a.eps));
            auto uu = [&](size_t i) { return a.F ? a.U[i] + a.F[i] : a.U[i]; };
            auto vv = [&](size_t i) { return a.F ? a.U[n + i] + a.F[n + i] : a.U[n + i]; };
            auto add = [&](int c, int xx, int yy, double v) {   // full flow U + F
                if (v == 0.0) return;
                unsafeAtomicAdd(&sfl[0][c][yy - y0 + 1][xx - x0 + 1], v);
                if (a.F) unsafeAtomicAdd(&sfl[1][c][yy - y0 + 1][xx - x0 + 1], v);
            };
            const double u0 = uu(g), v0 = vv(g);
            if (x < W - 1) {
                const double dxu = uu(g + 1) - u0, dxv = vv(g + 1) - v0;
                add(0, x + 1, y, 2.0 * dxu * gE); add(0, x, y, -2.0 * dxu * gE);
                add(1, x + 1, y, 2.0 * dxv * gE); add(1, x, y, -2.0 * dxv * gE);
            }
            if (y < H - 1) {
                const double dyu = uu(g + W) - u0, dyv = vv(g + W) - v0;
                add(0, x, y + 1, 2.0 * dyu * gE); add(0, x, y, -2.0 * dyu * gE);
                add(1, x, y + 1, 2.0 * dyv * gE); add(1, x, y, -2.0 * dyv * gE);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * 8 * 68; i += 256) {
        const int f = i / (8 * 68), r = i - f * (8 * 68), cy = r / 68, cx = r - cy * 68;
        const int gx = x0 - 2 + cx, gy = y0 - 2 + cy;
        const double v = simg[f][cy][cx];
        if (v != 0.0 && gx >= 0 && gx < W && gy >= 0 && gy < H)
            unsafeAtomicAdd((f ? a.gJ1w : a.gJ0) + (size_t)gy * W + gx, v);
    }
    for (int i = threadIdx.x; i < 2 * 2 * 6 * 66; i += 256) {
        const int f = i / (2 * 6 * 66), r = i - f * (2 * 6 * 66), c = r / (6 * 66), r2 = r - c * (6 * 66);
        const int cy = r2 / 66, cx = r2 - cy * 66;
        const int gx = x0 - 1 + cx, gy = y0 - 1 + cy;
        const double v = sfl[f][c][cy][cx];
        if (v != 0.0 && gx >= 0 && gx < W && gy >= 0 && gy < H)
            unsafeAtomicAdd((f ? a.gF : a.gU) + c * n + (size_t)gy * W + gx, v);
    }
}

// ------------------------------------------------- reverse refinement tile

namespace {

// The reverse of kh half sweeps needs a region one pixel wider than the
// forward's: within one reverse half sweep an error entering at the cut
// reaches the pixels of the other colour next to it (part b), so after kh
// of them it has moved kh + 1 pixels in.  The forward set-up's planes are
// dead once the coefficients are in registers, so the reverse's planes
// share their LDS; the state adjoint lives in the owners' registers (only
// a pixel's owner reads or writes it).
template <int TW, int TH, int KH>
struct BwdStepSmem {
    using F = dis_tile::RefineSmem<TW, TH, KH + 1>;
    static constexpr int RP = F::RHM * F::LP;
    union {
        F f;                            // forward set-up
        struct {
            double st_u[RP], st_v[RP];  // tape state before the half sweep being reversed
            double nu[RP], nv[RP];      // adjoints of the neighbour sums of the last reverse half sweep
            double acc[9][TW * TH];     // coefficient adjoints of the core pixels
        } r;
    };
};

}  // namespace

// WPE: waves per SIMD the register allocation must allow (4: two blocks of
// 512 threads per compute unit; both shapes in use fit without spilling)
template <int TW, int TH, int KH, int NT, int WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void k_bwd_step(const BwdStepArgs A) {
    constexpr int KG = KH + 1;
    using S = dis_tile::RefineSmem<TW, TH, KG>;
    using Shape = dis_tile::TileShape<TW, TH, NT, KG>;
    constexpr int LP = S::LP;
    constexpr int PPT = Shape::PPT;
    constexpr int NE = (S::RWM * S::RHM + NT - 1) / NT;   // region elements per thread
    __shared__ BwdStepSmem<TW, TH, KH> sm;
    const RefineArgs& a = A.ra;
    const int kh = __builtin_amdgcn_readfirstlane(A.j_hi - A.j_lo);
    const dis_tile::TileGeom g =
        dis_tile::tile_geom<TW, TH>(a.W, a.H, a.tiles_x, dis_xcd_tile(blockIdx.x, gridDim.x), kh + 1);
    const int W = g.W;
    const size_t n = (size_t)W * g.H;
    const int rx0 = g.rx0, ry0 = g.ry0, RW = g.RW, RH = g.RH;
    const int cx0 = g.cx0, cy0 = g.cy0, CW = g.cx1 - g.cx0, CH = g.cy1 - g.cy0;
    const double om1 = 1.0 - a.omega;

    dis_tile::TileCoef<PPT> C;
    double s_iu[Shape::NS][2], s_iv[Shape::NS][2];
    // the reverse steps below touch only pixels within kh of the core
    dis_tile::refine_setup<TW, TH, NT, KG>(a, g, sm.f, C, s_iu, s_iv, kh);
    __syncthreads();   // the set-up planes are dead from here on
    // The adjoint moves one pixel per reverse half sweep: after reverse step
    // r (of kh) the core's outputs still depend on pixels within kh - 1 - r
    // of it, so step r replays and reverses (a) pixels within kh - r and
    // gathers (b) into pixels within kh - 1 - r; the rest are skipped (the
    // tape supplies the forward states exactly, so the replay needs no
    // cone).  The core's results keep their bits.  Each owned pixel's
    // Chebyshev distance from the core goes to bits 8.. of its flag word.
    // State adjoint of the owned pixels, from gd_in (+ gadd).
    double ga_u[PPT][2], ga_v[PPT][2];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            ga_u[k][c] = ga_v[k][c] = 0.0;
            const int l = C.l[k][c];
            if (l < 0) continue;
            const int ly = l / LP, lx = l - ly * LP;
            const int x = rx0 + lx, y = ry0 + ly;
            const int d = max(max(max(cx0 - x, x - (g.cx1 - 1)), max(cy0 - y, y - (g.cy1 - 1))), 0);
            C.m[k][c] |= d << 8;
            const size_t gi = (size_t)y * W + x;
            double u = A.gd_in[gi], v = A.gd_in[n + gi];
            if (A.gadd) { u = u + A.gadd[gi]; v = v + A.gadd[n + gi]; }
            ga_u[k][c] = u;
            ga_v[k][c] = v;
        }
    }
    // coefficient adjoints of the core
    for (int i = threadIdx.x; i < CW * CH; i += NT) {
        const int yy = i / CW, xx = i - yy * CW;
        const size_t gi = (size_t)(cy0 + yy) * W + cx0 + xx;
#pragma unroll
        for (int q = 0; q < 9; ++q) sm.r.acc[q][yy * TW + xx] = A.acc_load ? A.acc[q * n + gi] : 0.0;
    }
    // the tape state before a half sweep, region-wide, through registers so
    // that the next one is in flight while the current one is reversed.  The
    // state before half sweep j differs from the one before j + 1 only at the
    // pixels half sweep j updated (colour j & 1), so after the first, full
    // state only those are fetched and replaced (colour: 0, 1, or -1 = all)
    double* st_u = sm.r.st_u;
    double* st_v = sm.r.st_v;
    double pu[NE], pv[NE];
    auto in_set = [&](int i, int colour) {
        if (i >= RW * RH) return false;
        if (colour < 0) return true;
        const int ly = i / RW, lx = i - ly * RW;
        return ((rx0 + lx + ry0 + ly) & 1) == colour;
    };
    auto fetch = [&](int j, int colour) {
        const int m = A.m0 + j;
        const double* tp = m ? A.tape + (size_t)m * 2 * n : nullptr;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int i = threadIdx.x + e * NT;
            pu[e] = pv[e] = 0.0;
            if (tp && in_set(i, colour)) {
                const int ly = i / RW, lx = i - ly * RW;
                const size_t gi = (size_t)(ry0 + ly) * W + rx0 + lx;
                pu[e] = tp[gi];
                pv[e] = tp[n + gi];
            }
        }
    };
    auto stash = [&](int colour) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int i = threadIdx.x + e * NT;
            if (in_set(i, colour)) {
                const int ly = i / RW, lx = i - ly * RW;
                st_u[ly * LP + lx] = pu[e];
                st_v[ly * LP + lx] = pv[e];
            }
        }
    };
    const int jhi = __builtin_amdgcn_readfirstlane(A.j_hi), jlo = __builtin_amdgcn_readfirstlane(A.j_lo);
    fetch(jhi - 1, -1);
    stash(-1);
    __syncthreads();
    // one reverse half sweep; the colour is a template constant so that the
    // per-pixel coefficient arrays stay in registers
    auto reverse = [&](auto colour, int j) {
        constexpr int c = decltype(colour)::value;   // the colour half sweep j updated
        if (j > jlo) fetch(j - 1, c ^ 1);             // half sweep j - 1 updated the other colour
        const int r = jhi - 1 - j;                    // reverse steps done before this one
        // (a) pixels of colour c: replay the update, then its adjoint
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int l = C.l[k][c];
            if (l < 0 || (C.m[k][c] >> 8) > kh - r) continue;
            const int msk = C.m[k][c];
            const int lr = (msk & 1) ? l + 1 : l, ll = (msk & 2) ? l - 1 : l;
            const int ld = (msk & 4) ? l + LP : l, lu = (msk & 8) ? l - LP : l;
            const double dup = st_u[l], dvp = st_v[l];
            const double dur = (msk & 1) ? st_u[lr] : 0.0, dul = (msk & 2) ? st_u[ll] : 0.0;
            const double dud = (msk & 4) ? st_u[ld] : 0.0, duu = (msk & 8) ? st_u[lu] : 0.0;
            const double dvr = (msk & 1) ? st_v[lr] : 0.0, dvl = (msk & 2) ? st_v[ll] : 0.0;
            const double dvd = (msk & 4) ? st_v[ld] : 0.0, dvu = (msk & 8) ? st_v[lu] : 0.0;
            const double wr = C.wr[k][c], wl = C.wl[k][c], wd = C.wd[k][c], wu = C.wu[k][c];
            const double A12 = C.a12[k][c], i1 = C.i1[k][c], i2 = C.i2[k][c];
            const double nu = ((wr * dur + wl * dul) + wd * dud) + wu * duu;
            const double r1 = (nu + C.c1[k][c]) - A12 * dvp;
            const double dun = om1 * dup + i1 * r1;
            const double nv = ((wr * dvr + wl * dvl) + wd * dvd) + wu * dvu;
            const double r2 = (nv + C.c2[k][c]) - A12 * dun;
            const double adv = ga_v[k][c];
            const double gr2 = i2 * adv;
            const double adu = ga_u[k][c] - A12 * gr2;
            const double gr1 = i1 * adu;
            const int ly = l / LP, lx = l - ly * LP;
            const int xx = rx0 + lx - cx0, yy = ry0 + ly - cy0;
            if (xx >= 0 && xx < CW && yy >= 0 && yy < CH) {
                const int q = yy * TW + xx;
                sm.r.acc[0][q] += r1 * adu;
                sm.r.acc[1][q] += r2 * adv;
                sm.r.acc[2][q] += gr1;
                sm.r.acc[3][q] += gr2;
                sm.r.acc[4][q] += -dun * gr2 - dvp * gr1;
                sm.r.acc[5][q] += dur * gr1 + dvr * gr2;
                sm.r.acc[6][q] += dul * gr1 + dvl * gr2;
                sm.r.acc[7][q] += dud * gr1 + dvd * gr2;
                sm.r.acc[8][q] += duu * gr1 + dvu * gr2;
            }
            ga_u[k][c] = om1 * adu;
            ga_v[k][c] = om1 * adv - A12 * gr1;
            sm.r.nu[l] = gr1;
            sm.r.nv[l] = gr2;
        }
        __syncthreads();
        // (b) pixels of the other colour collect what their neighbours'
        // updates owe them; the next state goes to LDS meanwhile
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int l = C.l[k][c ^ 1];
            if (l < 0 || (C.m[k][c ^ 1] >> 8) > kh - 1 - r) continue;
            const int msk = C.m[k][c ^ 1];
            double su = 0.0, sv = 0.0;
            if (msk & 1) { su += C.wr[k][c ^ 1] * sm.r.nu[l + 1]; sv += C.wr[k][c ^ 1] * sm.r.nv[l + 1]; }
            if (msk & 2) { su += C.wl[k][c ^ 1] * sm.r.nu[l - 1]; sv += C.wl[k][c ^ 1] * sm.r.nv[l - 1]; }
            if (msk & 4) { su += C.wd[k][c ^ 1] * sm.r.nu[l + LP]; sv += C.wd[k][c ^ 1] * sm.r.nv[l + LP]; }
            if (msk & 8) { su += C.wu[k][c ^ 1] * sm.r.nu[l - LP]; sv += C.wu[k][c ^ 1] * sm.r.nv[l - LP]; }
            ga_u[k][c ^ 1] += su;
            ga_v[k][c ^ 1] += sv;
        }
        if (j > jlo) stash(c ^ 1);
        __syncthreads();
    };
    for (int j = jhi - 1; j >= jlo; --j) {
        if (j & 1) reverse(std::integral_constant<int, 1>{}, j);
        else reverse(std::integral_constant<int, 0>{}, j);
    }

    // the core: coefficient adjoints, then per owned pixel the state adjoint
    // and the coefficients the linearisation adjoint reads (the smoothness
    // weight of the pixel's right edge, or of its lower edge in the last
    // column; core pixels see both neighbours whenever the image has them)
    for (int i = threadIdx.x; i < CW * CH; i += NT) {
        const int yy = i / CW, xx = i - yy * CW;
        const size_t gi = (size_t)(cy0 + yy) * W + cx0 + xx;
#pragma unroll
        for (int q = 0; q < 9; ++q) A.acc[q * n + gi] = sm.r.acc[q][yy * TW + xx];
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int l = C.l[k][c];
            if (l < 0) continue;
            const int ly = l / LP, lx = l - ly * LP;
            const int x = rx0 + lx, y = ry0 + ly;
            if (x < cx0 || x >= g.cx1 || y < cy0 || y >= g.cy1) continue;
            const size_t gi = (size_t)y * W + x;
            A.gd_out[gi] = ga_u[k][c];
            A.gd_out[n + gi] = ga_v[k][c];
            A.coef[n + gi] = C.i1[k][c];
            A.coef[2 * n + gi] = C.i2[k][c];
            A.coef[5 * n + gi] = x < W - 1 ? C.wr[k][c] : C.wd[k][c];
        }
    }
}

// ----------------------------------------------------------- densification

// Reverse of the warped frame J1w(x) = J1(x + Ud(x)) and of Eq. (3), in two
// passes so that no per-patch sum needs atomics.  Pass 1, per pixel: the
// dense flow's adjoint (plus the warped frame's, through the bilinear
// derivative) is stored for pass 2, and the residual adjoints of the
// covering patches go to J0 (a gather: plain add) and to J1's bilinear taps
// (atomics, spread over the frame).
// Covering patches of coordinate x along one axis: first index k0 (returned
// through the reference) and last regular index (the flush patch is extra).
__device__ __forceinline__ int bwd_cover(int x, int ps, int st, int nr, int& k0) {
    const int lo = x - ps + 1;
    k0 = lo <= 0 ? 0 : (lo + st - 1) / st;
    return min(x / st, nr - 1);
}

// The J1 adjoint a 64x4 block scatters lands near it wherever the flow and
// the covering patches' displacements are small: positions within
// DENS_WM pixels of the block (before the border clamp) are summed in LDS
// and added to memory once per cell; taps beyond go to memory directly.
constexpr int DENS_WM = 16, DENS_WW = 64 + 2 * DENS_WM, DENS_WH = 4 + 2 * DENS_WM;

__global__ __launch_bounds__(256) void k_bwd_densify(const DensBwdArgs a) {
    __shared__ double win[DENS_WH * DENS_WW];
    for (int i = threadIdx.x; i < DENS_WH * DENS_WW; i += 256) win[i] = 0.0;
    __syncthreads();
    const int W = a.W, H = a.H;
    const int wx0 = (int)blockIdx.x * 64 - DENS_WM, wy0 = (int)blockIdx.y * 4 - DENS_WM;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    auto scatter = [&](const Taps& t, double v) {
        const int X = t.fx - wx0, Y = t.fy - wy0;
        if (X >= 0 && Y >= 0 && X + 1 < DENS_WW && Y + 1 < DENS_WH) {
            double* c = win + Y * DENS_WW + X;
            if (v * t.w00 != 0.0) unsafeAtomicAdd(c, v * t.w00);
            if (v * t.w01 != 0.0) unsafeAtomicAdd(c + 1, v * t.w01);
            if (v * t.w10 != 0.0) unsafeAtomicAdd(c + DENS_WW, v * t.w10);
            if (v * t.w11 != 0.0) unsafeAtomicAdd(c + DENS_WW + 1, v * t.w11);
        } else {
            scatter_taps(a.gJ1, t, v);
        }
    };
    auto pixel = [&]() {
        const size_t g = (size_t)y * W + x, n = (size_t)W * H;
        const double Ux = a.Ud[g], Vx = a.Ud[n + g];
        double gUx = a.gUd[g], gVx = a.gUd[n + g];
        if (a.gJ1w) {
            const double gw = a.gJ1w[g];
            if (gw != 0.0) {
                const Taps t = taps_of(a.J1, W, H, (double)x + Ux, (double)y + Vx);
                gUx += gw * t.dx;
                gVx += gw * t.dy;
                scatter(t, gw);
            }
        }
        a.gq[g] = gUx;
        a.gq[n + g] = gVx;
        if (gUx == 0.0 && gVx == 0.0) return;
        const double Z = a.Z[g];
        const double j0 = a.J0[g];
        const int ps = a.ps, st = a.st;
        int kx0, ky0;
        const int kx1 = bwd_cover(x, ps, st, a.nrx, kx0), ky1 = bwd_cover(y, ps, st, a.nry, ky0);
        const bool fx = (a.nx > a.nrx) && (x >= W - ps), fy = (a.ny > a.nry) && (y >= H - ps);
        const int kyend = ky1 + (fy ? 1 : 0), kxend = kx1 + (fx ? 1 : 0);
        double gj0 = 0.0;
        for (int jy = ky0; jy <= kyend; ++jy) {
            const int ky = jy <= ky1 ? jy : a.nry;
            for (int jx = kx0; jx <= kxend; ++jx) {
                const int kx = jx <= kx1 ? jx : a.nrx;
                const double* P = a.patch + (size_t)(ky * a.nx + kx) * 4;
                const double u = P[0], v = P[1];
                const Taps t = taps_of(a.J1, W, H, (double)x + u, (double)y + v);
                const double d = a.raw_residual ? (t.val - j0) : ((t.val - j0) - P[2]);
                const double ad = fabs(d);
                const double gw = (gUx * (u - Ux) + gVx * (v - Vx)) / Z;
                const double gd = ad > 1.0 ? gw * (d > 0.0 ? -1.0 : 1.0) / (d * d) : 0.0;
                if (gd != 0.0) {
                    scatter(t, gd);
                    gj0 -= gd;
                }
            }
        }
        a.gJ0[g] += gj0;
    };
    if (x < W && y < H) pixel();
    __syncthreads();
    for (int i = threadIdx.x; i < DENS_WH * DENS_WW; i += 256) {
        const double v = win[i];
        if (v == 0.0) continue;
        const int Y = i / DENS_WW, X = i - Y * DENS_WW;
        unsafeAtomicAdd(a.gJ1 + (size_t)clampi(wy0 + Y, 0, H - 1) * W + clampi(wx0 + X, 0, W - 1), v);
    }
}

// Pass 2, per patch (16 lanes, a lane's pixels strided by 16): the patch's
// sums over its template square of the displacement adjoints (weight times
// the flow adjoint over Z, and the residual adjoint times the bilinear
// derivative) and of the mean residual's adjoint; one plain add per entry.
__global__ __launch_bounds__(256) void k_bwd_densify_patch(const DensBwdArgs a) {
    const int W = a.W, H = a.H;
    const size_t n = (size_t)W * H;
    const int N = a.nx * a.ny;
    const int lane = threadIdx.x & 15;
    int i = (int)((blockIdx.x * 256u + threadIdx.x) >> 4);
    const bool valid = i < N;
    if (!valid) i = N - 1;          // idle lanes shadow the last patch and store nothing
    const int ps = a.ps;
    const int ky = i / a.nx, kx = i - ky * a.nx;
    const int x0 = kx < a.nrx ? kx * a.st : W - ps;
    const int y0 = ky < a.nry ? ky * a.st : H - ps;
    const double* P = a.patch + (size_t)i * 4;
    const double u = P[0], v = P[1], md = P[2];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int p = lane; p < ps * ps; p += 16) {
        const int py = p / ps, px = p - py * ps;
        const int x = x0 + px, y = y0 + py;
        const size_t g = (size_t)y * W + x;
        const double gUx = a.gq[g], gVx = a.gq[n + g];
        if (gUx == 0.0 && gVx == 0.0) continue;
        const double Ux = a.Ud[g], Vx = a.Ud[n + g];
        const double Z = a.Z[g];
        const double j0 = a.J0[g];
        const Taps t = taps_of(a.J1, W, H, (double)x + u, (double)y + v);
        const double d = a.raw_residual ? (t.val - j0) : ((t.val - j0) - md);
        const double ad = fabs(d);
        const double wgt = 1.0 / fmax(1.0, ad);
        s0 += gUx * wgt / Z;
        s1 += gVx * wgt / Z;
        const double gw = (gUx * (u - Ux) + gVx * (v - Vx)) / Z;
        const double gd = ad > 1.0 ? gw * (d > 0.0 ? -1.0 : 1.0) / (d * d) : 0.0;
        s0 += gd * t.dx;
        s1 += gd * t.dy;
        if (!a.raw_residual) s2 -= gd;
    }
    s0 = lane_sum<16>(s0);
    s1 = lane_sum<16>(s1);
    s2 = lane_sum<16>(s2);
    if (valid && lane == 0) {
        double* gP = a.gP + (size_t)i * 4;
        gP[0] += s0;
        gP[1] += s1;
        gP[2] += s2;
    }
}

// ------------------------------------------------------------------- pyramid

// I -> J_s = 255 * (2^s x 2^s box mean): each input pixel collects its
// level pixels' adjoints times 4^-s.
__global__ __launch_bounds__(256) void k_bwd_pyramid(const PyrBwdArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.W || y >= a.H) return;
    double g0 = 0.0, g1 = 0.0, sc = 1.0;
    for (int s = 0; s <= a.ss; ++s) {
        if (s >= a.sf) {
            const int xs = x >> s, ys = y >> s;
            if (xs < a.ws[s] && ys < a.hs[s]) {
                const size_t i = (size_t)ys * a.ws[s] + xs;
                g0 += sc * a.gJ0[s][i];
                g1 += sc * a.gJ1[s][i];
            }
        }
        sc *= 0.25;
    }
    const size_t g = (size_t)y * a.W + x;
    if (a.out_f64) {
        ((double*)a.gI0)[g] = 255.0 * g0;
        ((double*)a.gI1)[g] = 255.0 * g1;
    } else {
        ((float*)a.gI0)[g] = (float)(255.0 * g0);
        ((float*)a.gI1)[g] = (float)(255.0 * g1);
    }
}

// ------------------------------------------------------------------- search

// Reverse of the inverse-compositional search of one block of patches
// (LPP lanes per patch, as in the forward).  The forward iterates are
// recomputed and kept in LDS, then the theta_it updates
// u <- u - M b(u) (M = (H + lambda I)^-1) are reversed; gradients reach the
// taps of J1, the template and its Sobel gradients in J0, and, through the
// initialisation 2 U_{s+1}(c/2), the coarser flow.
//
// Each patch owns a WIN x WIN LDS window of J1 positions (before the border
// clamp): it collects the patch's J1 adjoint and, with VW, also holds the J1
// values the warps read, so that both passes over the iterates sample LDS
// instead of gathering from memory.  With VW the window is placed before the
// recomputation, around the initial and the final displacement (the
// iterates usually move between the two); without it, around the recomputed
// iterates.  A tap outside the window reads and scatters through global
// memory, with the same arithmetic.
template <int PS, int LPP, bool VW>
__device__ __forceinline__ void bwd_search_block(const SearchBwdArgs& A) {
    constexpr int NP = PS * PS;
    constexpr int PPL = (NP + LPP - 1) / LPP;
    constexpr int GROUPS = 256 / LPP;
    // dynamic LDS: [GROUPS][iters + 1][2] iterates, then per group the
    // adjoint window and (VW) the value window, WIN * WIN cells each
    extern __shared__ double s_dyn[];
    const SearchArgs& a = A.sa;
    const int W = a.W, H = a.H;
    const int lane = threadIdx.x & (LPP - 1);
    const int grp = threadIdx.x / LPP;
    const int N = a.nx * a.ny;
    const int WIN = A.win;
    auto* s_u = dis_lds(s_dyn);
    double* win = s_dyn + (size_t)GROUPS * (a.iters + 1) * 2 + (size_t)grp * (VW ? 2 : 1) * WIN * WIN;
    auto* vwin = dis_lds(win + WIN * WIN);
    int pi = (int)((blockIdx.x * 256u + threadIdx.x) / LPP);
    const bool valid = pi < N;
    if (!valid) pi = N - 1;
    const int ky = pi / a.nx, kx = pi - ky * a.nx;
    const int x0 = kx < a.nrx ? kx * a.st : W - PS;
    const int y0 = ky < a.nry ? ky * a.st : H - PS;
    double qx = 0.0, qy = 0.0, ui = 0.0, vi = 0.0;
    if (a.Un) {
        const double c = 0.5 * (PS - 1);
        qx = (double)x0 + c;
        qy = (double)y0 + c;
        if (a.centre_map) { qx = (qx + 0.5) / 2.0 - 0.5; qy = (qy + 0.5) / 2.0 - 0.5; }
        else { qx = qx / 2.0; qy = qy / 2.0; }
        ui = 2.0 * taps_of(a.Un, a.Wn, a.Hn, qx, qy).val;
        vi = 2.0 * taps_of(a.Un + (size_t)a.Wn * a.Hn, a.Wn, a.Hn, qx, qy).val;
    }
    const auto* J0 = dis_global(a.J0);
    const auto* J1 = dis_global(a.J1);
    // pixels of this lane: p = lane + k * LPP
    double T[PPL], gx[PPL], gy[PPL];
    double sgx_l = 0.0, sgy_l = 0.0, h11_l = 0.0, h12_l = 0.0, h22_l = 0.0;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int p = lane + k * LPP;
        T[k] = gx[k] = gy[k] = 0.0;
        if (p < NP) {
            const int py = p / PS, px = p - py * PS;
            const int x = x0 + px, y = y0 + py;
            const int xm = max(x - 1, 0), xp = min(x + 1, W - 1), ym = max(y - 1, 0), yp = min(y + 1, H - 1);
            T[k] = J0[y * W + x];
            const double dm = J0[ym * W + xp] - J0[ym * W + xm];
            const double d0 = J0[y * W + xp] - J0[y * W + xm];
            const double dp = J0[yp * W + xp] - J0[yp * W + xm];
            gx[k] = ((dm + 2.0 * d0) + dp) / 8.0;
            const double em = J0[yp * W + xm] - J0[ym * W + xm];
            const double e0 = J0[yp * W + x] - J0[ym * W + x];
            const double ep = J0[yp * W + xp] - J0[ym * W + xp];
            gy[k] = ((em + 2.0 * e0) + ep) / 8.0;
        }
        sgx_l += gx[k]; sgy_l += gy[k];
        h11_l += gx[k] * gx[k]; h12_l += gx[k] * gy[k]; h22_l += gy[k] * gy[k];
    }
    auto red = [&](double v) { return lane_sum<LPP>(v); };
    const double sgx = red(sgx_l), sgy = red(sgy_l);
    const double a11 = red(h11_l) + a.lam, a12 = red(h12_l), a22 = red(h22_l) + a.lam;
    const double idet = 1.0 / (a11 * a22 - a12 * a12);
    const double m11 = a22 * idet, m12 = -a12 * idet, m22 = a11 * idet;
    const double inv_n = 1.0 / (double)NP;
    const double lim = (double)(W + H + 2 * PS + 4);
    const auto* P = dis_global(a.patch) + (size_t)pi * 4;
    const double uf = P[0], vf = P[1];
    const bool reset = P[3] > (double)PS;
    const auto* gP = dis_global(A.gP) + (size_t)pi * 4;
    double gu = gP[0], gv = gP[1];
    const double gmd = gP[2];
    const bool iterate = !reset && a.iters > 0;
    double gT[PPL], ggx[PPL], ggy[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) gT[k] = ggx[k] = ggy[k] = 0.0;

    // integer part of a warp position (the displacement clamp included)
    auto ifloor = [&](double u) { return (int)fmin(fmax(floor(u), -lim), lim); };
    // window origin: the integer extent [lo, hi] of the warps in the middle,
    // with room for the patch, a pixel before it and two after it (a
    // position whose fraction rounds up to the next integer)
    int wx0 = 0, wy0 = 0;
    auto place = [&](int xlo, int xhi, int ylo, int yhi) {
        wx0 = x0 + xlo - 1 - max(WIN - (PS + 3) - (xhi - xlo), 0) / 2;
        wy0 = y0 + ylo - 1 - max(WIN - (PS + 3) - (yhi - ylo), 0) / 2;
    };
    // whether every tap of the warp at displacement (u, v) falls inside the
    // window: a tap's floor lies 0 or 1 (a fraction rounding up) past
    // x0 + px + floor(u), so floor(u) within [wx0 - x0, wx0 - x0 + WIN - PS
    // - 2] suffices; the same in y.  Uniform over the patch's lanes, which
    // hold the same (u, v).
    auto inside = [&](double u, double v) {
        const int iu = ifloor(u) - (wx0 - x0), iv = ifloor(v) - (wy0 - y0);
        return iu >= 0 && iu <= WIN - PS - 2 && iv >= 0 && iv <= WIN - PS - 2;
    };
    // one bilinear sample of J1 (from the value window when inw): taps
    // (floor before any clamp, fractions), value and its partial
    // derivatives, as taps_of computes them
    struct Tap { int fx, fy; double ax, ay; };
    auto sample = [&](bool inw, double x, double y, Tap& t, double& val, double& dx, double& dy) {
        const double xf = floor(x), yf = floor(y);
        t.ax = x - xf;
        t.ay = y - yf;
        t.fx = (int)xf;
        t.fy = (int)yf;
        double va, vb, vc, vd;
        if (VW && inw) {
            const auto* c = vwin + (t.fy - wy0) * WIN + (t.fx - wx0);
            va = c[0]; vb = c[1]; vc = c[WIN]; vd = c[WIN + 1];
        } else {
            const int ix0 = clampi(t.fx, 0, W - 1), ix1 = clampi(t.fx + 1, 0, W - 1);
            const int iy0 = clampi(t.fy, 0, H - 1), iy1 = clampi(t.fy + 1, 0, H - 1);
            va = J1[iy0 * W + ix0]; vb = J1[iy0 * W + ix1];
            vc = J1[iy1 * W + ix0]; vd = J1[iy1 * W + ix1];
        }
        const double ax = t.ax, ay = t.ay;
        const double top = (1.0 - ax) * va + ax * vb, bot = (1.0 - ax) * vc + ax * vd;
        val = (1.0 - ay) * top + ay * bot;
        dx = (1.0 - ay) * (vb - va) + ay * (vd - vc);
        dy = bot - top;
    };
    // residual of the patch at displacement (u, v): d_p, its derivatives, taps
    auto warp = [&](bool inw, double u, double v, double (&d)[PPL], double (&dx)[PPL], double (&dy)[PPL],
                    Tap (&tp)[PPL]) {
        const double fu = floor(u), fv = floor(v);
        const double cu = fmin(fmax(fu, -lim), lim) + (u - fu), cv = fmin(fmax(fv, -lim), lim) + (v - fv);
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int p = lane + k * LPP;
            d[k] = dx[k] = dy[k] = 0.0;
            if (p < NP) {
                const int py = p / PS, px = p - py * PS;
                double val;
                sample(inw, (double)(x0 + px) + cu, (double)(y0 + py) + cv, tp[k], val, dx[k], dy[k]);
                d[k] = val - T[k];
            }
        }
    };
    // clear the adjoint window (and fill the value window) at the origin
    auto fill = [&]() {
        for (int i = lane; i < WIN * WIN; i += LPP) {
            win[i] = 0.0;
            if (VW) {
                const int Y = i / WIN, X = i - Y * WIN;
                vwin[i] = J1[(size_t)clampi(wy0 + Y, 0, H - 1) * W + clampi(wx0 + X, 0, W - 1)];
            }
        }
        __builtin_amdgcn_wave_barrier();
    };

    if (VW) {
        const int fxu = ifloor(uf), fyv = ifloor(vf);
        const int ixa = iterate ? ifloor(ui) : fxu, iya = iterate ? ifloor(vi) : fyv;
        place(min(ixa, fxu), max(ixa, fxu), min(iya, fyv), max(iya, fyv));
        fill();
    }
    // forward iterates u_0 .. u_iters (every lane of the patch holds the same
    // bits of (u, v): the butterfly sums are commutative), and the integer
    // extent of every warp the reverse touches
    auto* su_ = s_u + (size_t)grp * (a.iters + 1) * 2;
    int ix_lo = ifloor(uf), ix_hi = ix_lo, iy_lo = ifloor(vf), iy_hi = iy_lo;
    double d[PPL], dqx[PPL], dqy[PPL];
    Tap tp[PPL];
    if (iterate) {
        double u = ui, v = vi;
        for (int it = 0; it < a.iters; ++it) {
            su_[2 * it] = u;
            su_[2 * it + 1] = v;
            const int iu = ifloor(u), iv = ifloor(v);
            ix_lo = min(ix_lo, iu); ix_hi = max(ix_hi, iu);
            iy_lo = min(iy_lo, iv); iy_hi = max(iy_hi, iv);
            warp(VW && inside(u, v), u, v, d, dqx, dqy, tp);
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int k = 0; k < PPL; ++k) { s0 += d[k]; s1 += gx[k] * d[k]; s2 += gy[k] * d[k]; }
            const double md = red(s0) * inv_n;
            const double b1 = red(s1) - md * sgx, b2 = red(s2) - md * sgy;
            u = u - (m11 * b1 + m12 * b2);
            v = v - (m12 * b1 + m22 * b2);
        }
    }
    if (!VW) {
        place(ix_lo, ix_hi, iy_lo, iy_hi);
        fill();
    }
    // the J1 adjoint of one tap set: into the window when the warp's taps
    // all fall inside it (inw), else straight to memory
    auto scatter_j1 = [&](bool inw, int k, double val) {
        const Tap& t = tp[k];
        const double ax = t.ax, ay = t.ay;
        const double w00 = (1.0 - ay) * (1.0 - ax), w01 = (1.0 - ay) * ax, w10 = ay * (1.0 - ax), w11 = ay * ax;
        if (inw) {
            double* c = win + (t.fy - wy0) * WIN + (t.fx - wx0);
            unsafeAtomicAdd(c, val * w00);
            unsafeAtomicAdd(c + 1, val * w01);
            unsafeAtomicAdd(c + WIN, val * w10);
            unsafeAtomicAdd(c + WIN + 1, val * w11);
        } else {
            const int ix0 = clampi(t.fx, 0, W - 1), ix1 = clampi(t.fx + 1, 0, W - 1);
            const int iy0 = clampi(t.fy, 0, H - 1), iy1 = clampi(t.fy + 1, 0, H - 1);
            atom(A.gJ1 + iy0 * W + ix0, val * w00);
            atom(A.gJ1 + iy0 * W + ix1, val * w01);
            atom(A.gJ1 + iy1 * W + ix0, val * w10);
            atom(A.gJ1 + iy1 * W + ix1, val * w11);
        }
    };

    // mean residual at the final displacement (used by the densification)
    if (gmd != 0.0) {
        const bool inw = inside(uf, vf);
        warp(VW && inw, uf, vf, d, dqx, dqy, tp);
        const double q = gmd * inv_n;
        double su = 0.0, sv = 0.0;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int p = lane + k * LPP;
            if (p < NP) {
                su += q * dqx[k];
                sv += q * dqy[k];
                if (valid) scatter_j1(inw, k, q);
                gT[k] -= q;
            }
        }
        gu += red(su);
        gv += red(sv);
    }
    double gui = gu, gvi = gv;
    if (iterate) {
        double H11 = 0.0, H12 = 0.0, H21 = 0.0, H22 = 0.0;   // adjoint of H
        for (int it = a.iters - 1; it >= 0; --it) {
            const double uk = su_[2 * it], vk = su_[2 * it + 1];
            const bool inw = inside(uk, vk);
            warp(VW && inw, uk, vk, d, dqx, dqy, tp);
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int k = 0; k < PPL; ++k) { s0 += d[k]; s1 += gx[k] * d[k]; s2 += gy[k] * d[k]; }
            const double md = red(s0) * inv_n;
            const double b1 = red(s1) - md * sgx, b2 = red(s2) - md * sgy;
            // u_{k+1} = u_k - Delta, Delta = M b
            const double Dl1 = -gu, Dl2 = -gv;                      // adjoint of Delta
            const double bb1 = m11 * Dl1 + m12 * Dl2, bb2 = m12 * Dl1 + m22 * Dl2;   // adjoint of b
            const double D1 = m11 * b1 + m12 * b2, D2 = m12 * b1 + m22 * b2;
            H11 -= bb1 * D1; H12 -= bb1 * D2; H21 -= bb2 * D1; H22 -= bb2 * D2;
            double su = 0.0, sv = 0.0;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                const int p = lane + k * LPP;
                if (p < NP) {
                    // b = sum g (d - md): d(b)/d(d_p) = g_p - sum(g)/n
                    const double dd = bb1 * (gx[k] - sgx * inv_n) + bb2 * (gy[k] - sgy * inv_n);
                    ggx[k] += bb1 * (d[k] - md);
                    ggy[k] += bb2 * (d[k] - md);
                    gT[k] -= dd;
                    su += dd * dqx[k];
                    sv += dd * dqy[k];
                    if (valid) scatter_j1(inw, k, dd);
                }
            }
            gu += red(su);
            gv += red(sv);
        }
        gui = gu;
        gvi = gv;
        // H = sum g g^T + lambda I
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            ggx[k] += (H11 + H11) * gx[k] + (H12 + H21) * gy[k];
            ggy[k] += (H12 + H21) * gx[k] + (H22 + H22) * gy[k];
        }
    }
    // the window, with the taps' clamp to the image
    __builtin_amdgcn_wave_barrier();
    if (valid) {
        for (int i = lane; i < WIN * WIN; i += LPP) {
            const int Y = i / WIN, X = i - Y * WIN;
            const double v = win[i];
            if (v != 0.0) unsafeAtomicAdd(A.gJ1 + (size_t)clampi(wy0 + Y, 0, H - 1) * W + clampi(wx0 + X, 0, W - 1), v);
        }
    }
    // template and Sobel/8 gradients -> J0, through the same window (cells
    // x0 - 1 .. x0 + PS, y0 - 1 .. y0 + PS before the border clamp)
    __builtin_amdgcn_wave_barrier();
    const int jx0 = x0 - 1, jy0 = y0 - 1, JW = PS + 2;
    for (int i = lane; i < JW * JW; i += LPP) win[(i / JW) * WIN + (i % JW)] = 0.0;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int p = lane + k * LPP;
        if (p >= NP) continue;
        const int py = p / PS, px = p - py * PS;
        double* c = win + (py + 1) * WIN + (px + 1);   // the pixel itself
        const double ax = ggx[k] / 8.0, ay = ggy[k] / 8.0;
        unsafeAtomicAdd(c, gT[k]);
        unsafeAtomicAdd(c - WIN + 1, ax); unsafeAtomicAdd(c - WIN - 1, -ax);
        unsafeAtomicAdd(c + 1, 2.0 * ax); unsafeAtomicAdd(c - 1, -2.0 * ax);
        unsafeAtomicAdd(c + WIN + 1, ax); unsafeAtomicAdd(c + WIN - 1, -ax);
        unsafeAtomicAdd(c + WIN - 1, ay); unsafeAtomicAdd(c - WIN - 1, -ay);
        unsafeAtomicAdd(c + WIN, 2.0 * ay); unsafeAtomicAdd(c - WIN, -2.0 * ay);
        unsafeAtomicAdd(c + WIN + 1, ay); unsafeAtomicAdd(c - WIN + 1, -ay);
    }
    __builtin_amdgcn_wave_barrier();
    if (valid) {
        for (int i = lane; i < JW * JW; i += LPP) {
            const int Y = i / JW, X = i - Y * JW;
            const double v = win[Y * WIN + X];
            if (v != 0.0)
                unsafeAtomicAdd(A.gJ0 + (size_t)clampi(jy0 + Y, 0, H - 1) * W + clampi(jx0 + X, 0, W - 1), v);
        }
    }
    if (!valid) return;
    // initialisation u_init = 2 U_{s+1}(q)
    if (a.Un && lane == 0) {
        const Taps t = taps_of(nullptr, a.Wn, a.Hn, qx, qy);
        scatter_taps(A.gUn, t, 2.0 * gui);
        scatter_taps(A.gUn + (size_t)a.Wn * a.Hn, t, 2.0 * gvi);
    }
}

// Up to 8x8 patches the reverse search fits two waves per SIMD in 256
// registers, which hides more of its latency than one wave with all the
// registers it asks for, and keeps its J1 values in the LDS window; larger
// patches sample J1 in memory (two windows would not fit 64 KB of LDS).
template <int PS, int LPP>
__global__ __launch_bounds__(256) void k_bwd_search(const SearchBwdArgs A) {
    bwd_search_block<PS, LPP, false>(A);
}

template <int PS, int LPP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_bwd_search_w2(const SearchBwdArgs A) {
    bwd_search_block<PS, LPP, true>(A);
}

// ------------------------------------------------------------ kernel table

const void* dis_kernel_bzero() { return (const void*)&k_bzero; }
const void* dis_kernel_bzero_list() { return (const void*)&k_bzero_list; }
// reverse refinement tiles: core width, height and half sweeps per launch
// (and the waves per SIMD their registers allow)
#define DIS_BWD_STEP_SHAPES(X) X(8, 8, 10, 4) X(16, 16, 5, 4)
const void* dis_kernel_bwd_step(int shape) {
    int i = 0;
#define X(tw, th, kh, wpe) if (shape == i++) return (const void*)&k_bwd_step<tw, th, kh, DIS_BWD_THREADS, wpe>;
    DIS_BWD_STEP_SHAPES(X)
#undef X
    return nullptr;
}
int dis_bwd_step_shape(int shape, int* tw, int* th, int* kh) {
    int i = 0;
#define X(w_, h_, k_, wpe) if (shape == i++) { *tw = w_; *th = h_; *kh = k_; return 1; }
    DIS_BWD_STEP_SHAPES(X)
#undef X
    return 0;
}
const void* dis_kernel_bcopy() { return (const void*)&k_bcopy; }
const void* dis_kernel_baxpy() { return (const void*)&k_baxpy; }
const void* dis_kernel_bwd_upsample() { return (const void*)&k_bwd_upsample; }
const void* dis_kernel_bwd_coef() { return (const void*)&k_bwd_coef; }
const void* dis_kernel_bwd_coef2() { return (const void*)&k_bwd_coef2; }
const void* dis_kernel_bwd_sweep_a() { return (const void*)&k_bwd_sweep_a; }
const void* dis_kernel_bwd_sweep_b() { return (const void*)&k_bwd_sweep_b; }
const void* dis_kernel_bwd_lin_ws() { return (const void*)&k_bwd_lin_ws; }
const void* dis_kernel_bwd_densify_patch() { return (const void*)&k_bwd_densify_patch; }
const void* dis_kernel_bwd_densify() { return (const void*)&k_bwd_densify; }
const void* dis_kernel_bwd_pyramid() { return (const void*)&k_bwd_pyramid; }

#define DIS_BWD_SEARCH_CASE(PS_) \
    if (ps == PS_) return PS_ <= 8 ? (const void*)&k_bwd_search_w2<PS_, 16> : (const void*)&k_bwd_search<PS_, 16>;
int dis_bwd_search_windows(int ps) { return ps <= 8 ? 2 : 1; }
const void* dis_kernel_bwd_search(int ps) {
    DIS_BWD_SEARCH_CASE(4) DIS_BWD_SEARCH_CASE(6) DIS_BWD_SEARCH_CASE(8) DIS_BWD_SEARCH_CASE(10)
    DIS_BWD_SEARCH_CASE(12) DIS_BWD_SEARCH_CASE(14) DIS_BWD_SEARCH_CASE(16)
    return nullptr;
}
