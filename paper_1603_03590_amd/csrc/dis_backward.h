// Argument blocks of the adjoint kernels (one struct per kernel, by value).
#pragma once
#include <stddef.h>
#include "dis_internal.h"

struct BZeroArgs {
    double* p;
    size_t n;
};

// Clear up to 8 buffers in one launch: block b clears part of the buffer
// whose block range [start[i], start[i+1]) holds b.
struct BZeroList {
    double* p[8];
    size_t n[8];
    int start[9];
    int cnt;
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

// Reverse of the half sweeps j_hi-1 .. j_lo of one fixed-point step of the
// refinement on one tile (core grown by j_hi - j_lo + 1 on every cut side):
// the step's coefficients are recomputed as in the forward tile, the states
// before each half sweep come from the tape, the state adjoint lives in the
// owning threads' registers.
// Core pixels write the adjoint of the state before half sweep j_lo, their 9
// coefficient adjoints (summed over the step's half sweeps) and the
// coefficients the linearisation adjoint needs.
struct BwdStepArgs {
    RefineArgs ra;          // the forward step: U = Ud, J0, J1w, dUf = frozen increment (null = zero), tiles_x
    const double* tape;     // state before half sweep j at tape + (m0 + j) * 2 W H; zero when m0 + j == 0
    int m0;
    int j_lo, j_hi;         // j_hi - j_lo <= the shape's half sweeps per launch
    const double* gd_in;    // adjoint of the state after half sweep j_hi - 1 [2][H][W]
    const double* gadd;     // added to gd_in, or null
    double* gd_out;         // adjoint of the state before half sweep j_lo
    double* coef;           // [6][H][W]: planes 1, 2, 5 (omega/(A11+S), omega/(A22+S), ws) written
    double* acc;            // [9][H][W] coefficient adjoints
    int acc_load;           // 1: continue the sums already in acc
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
    double* gq;             // [2][H][W] scratch: the flow adjoint pass 1 hands to pass 2
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
    int win;                // cells per side of each patch's LDS window(s), at least PS + 3; taps outside it go through memory
};

const void* dis_kernel_bzero();
const void* dis_kernel_bzero_list();
// reverse refinement tiles, by shape id: core width and height and the most
// half sweeps one launch reverses (0: 8x8 cores over up to 10 half sweeps,
// 1: 16x16 cores over up to 5); 512 threads, two blocks per compute unit;
// null / 0 past the last id
const void* dis_kernel_bwd_step(int shape);
int dis_bwd_step_shape(int shape, int* tw, int* th, int* kh);
#define DIS_BWD_THREADS 512
const void* dis_kernel_bcopy();
const void* dis_kernel_baxpy();
const void* dis_kernel_bwd_upsample();
const void* dis_kernel_bwd_coef();
const void* dis_kernel_bwd_coef2();
const void* dis_kernel_bwd_sweep_a();
const void* dis_kernel_bwd_sweep_b();
const void* dis_kernel_bwd_lin_ws();
const void* dis_kernel_bwd_densify();         // pass 1, per pixel
const void* dis_kernel_bwd_densify_patch();   // pass 2, 16 lanes per patch
const void* dis_kernel_bwd_pyramid();
const void* dis_kernel_bwd_search(int ps);
// LDS windows per patch of that kernel: 2 (adjoint and J1 values) or 1
int dis_bwd_search_windows(int ps);
