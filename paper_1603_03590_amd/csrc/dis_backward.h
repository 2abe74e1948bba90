// Argument blocks of the adjoint kernels (one struct per kernel, by value).
#pragma once
#include <stddef.h>
#include "dis_internal.h"

struct BZeroArgs {
    double* p;
    size_t n;
};

struct BCopyArgs {
    double* dst;
    const double* src;
    double* dst2;       // optional second destination (copy only)
    size_t n;
};

// Adjoint of the upscaling: gF (caller's [2][H][W]) -> gU ([2][Hs][Ws]).
struct UpsBwdArgs {
    const void* gF;
    int g_f64;
    int W, H;
    double f;
    int centre_map;
    double* gU;
    int Ws, Hs;
};

// One fixed-point step of the refinement, for its coefficient kernels.
struct RefBwdArgs {
    const double* U;        // densified flow Ud [2][H][W]
    const double* F;        // frozen increment of this step (null = zero)
    const double* J0;
    const double* J1w;
    double* coef;           // [6][H][W]: A12, om/(A11+S), om/(A22+S), c1, c2, ws
    double* acc;            // [9][H][W] coefficient adjoints from the sweeps
    double* edge;           // [4][H][W] edge-weight adjoints seen from each endpoint (r, l, d, u)
    double* gU;             // += adjoint of Ud
    double* gF;             // += adjoint of F
    double* gJ0;            // += adjoint of J0 (level)
    double* gJ1w;           // += adjoint of the warped frame
    int W, H;
    double delta, gamma, alpha, omega, eps;
};

// Reverse of one red-black half sweep.
struct SweepBwdArgs {
    const double* state;    // state before the half sweep [2][H][W] (null = zero)
    const double* coef;
    double* gd;             // adjoint of the state [2][H][W]
    double* gn;             // adjoints of the neighbour sums [2][H][W]
    double* acc;
    int W, H;
    int colour;
    double omega;
};

struct DensBwdArgs {
    const double* J0;
    const double* J1;
    int W, H;
    const double* patch;
    int ps, st, nrx, nry, nx, ny;
    int raw_residual;
    const double* Ud;
    const double* Z;
    const double* gUd;      // adjoint of the densified flow
    const double* gJ1w;     // adjoint of the warped frame, or null
    double* gJ0;
    double* gJ1;
    double* gP;             // [N][4]: adjoints of u, v, mean residual
};

struct PyrBwdArgs {
    const double* gJ0[DIS_MAXL];
    const double* gJ1[DIS_MAXL];
    int ws[DIS_MAXL], hs[DIS_MAXL];
    int sf, ss, W, H;
    int out_f64;
    void* gI0;
    void* gI1;
};

struct SearchBwdArgs {
    SearchArgs sa;
    const double* gP;
    double* gJ0;
    double* gJ1;
    double* gUn;            // adjoint of the coarser flow (null on the coarsest level)
};

const void* dis_kernel_bzero();
const void* dis_kernel_bcopy();
const void* dis_kernel_baxpy();
const void* dis_kernel_bwd_upsample();
const void* dis_kernel_bwd_coef();
const void* dis_kernel_bwd_coef2();
const void* dis_kernel_bwd_sweep_a();
const void* dis_kernel_bwd_sweep_b();
const void* dis_kernel_bwd_lin();
const void* dis_kernel_bwd_ws();
const void* dis_kernel_bwd_densify();
const void* dis_kernel_bwd_pyramid();
const void* dis_kernel_bwd_search(int ps);
