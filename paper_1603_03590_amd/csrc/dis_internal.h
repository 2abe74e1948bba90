// Launch-argument blocks shared by the host library and the HIP kernels.
// Every kernel takes exactly one of these structs by value.  All planes are
// dense row-major float64 arrays (pitch = width) owned by the handle, except
// the caller's frames and flow.
#pragma once
#include <stdint.h>

#define DIS_MAXL 16   // pyramid levels a handle can hold
#define DIS_KMAX 10   // red-black half sweeps one refinement launch can fuse
#define DIS_LEVEL_TILE 0   // refinement tile id used inside the persistent level kernel by default
// the refinement tile the persistent level kernel uses when `tile` is asked
// for: tile 1 (16x16 on 256 threads) with the row-owned search, else tile 0
// (32x16 on 256 threads)
inline int dis_level_tile(int tile, bool rows) { return (rows && tile == 1) ? 1 : DIS_LEVEL_TILE; }

// Pyramid: from level `a` (the caller's frames when a == 0) compute the
// 2x2-box levels a+1 .. a+nlev (nlev <= 5) in one pass over 32x32 tiles.
struct PyrArgs {
    const void* src[2];     // frame 0 / frame 1 of level a
    int src_kind;           // 0 = float64 plane, 1 = float32 frame, 2 = float64 frame
    int src_pitch;          // elements
    double scale;           // 255 for frames, 1 for planes
    long long src_cstride;  // elements between the colour channels of src
    int nc;                 // channels (grid y = 2 nc: frame = y & 1, channel = y >> 1)
    int a, nlev;
    int w0, h0;             // size of level a
    int tiles_x;
    double* lvl0[2];        // receives the scaled level a when non-null
    double* dst[2][6];      // dst[f][k]: level a+k, or null when not kept
    int ws[6], hs[6];
    int* zero;              // block 0 clears these ints (queue state of the level launches)
    int nzero;
};

// 256x32 tiles (512-thread blocks) of level a a pyramid pass covers
#define DIS_PYR_THREADS 512
inline int dis_pyramid_tiles(const PyrArgs& pa) { return pa.tiles_x * ((pa.h0 + 31) / 32); }

// output rows of one upscaling block (256 columns wide) of a W x H flow: 16
// from a megapixel up (fewer tap rounds per pixel), else 8 (more blocks in
// flight for a short launch); and the block rows of the flow
inline int dis_upsample_rows(int W, int H) { return (long long)W * H >= (1 << 20) ? 16 : 8; }
inline int dis_upsample_blocks_y(int W, int H) { return (H + dis_upsample_rows(W, H) - 1) / dis_upsample_rows(W, H); }

// Inverse search on one level: grid, initialisation, Gauss-Newton, reset,
// final residual mean.
struct SearchArgs {
    const double* J0;
    const double* J1;
    int W, H;
    const double* Un;       // coarser flow [2][Hn][Wn]; null on the coarsest level
    int Wn, Hn;
    int st, nrx, nry, nx, ny;   // stride; regular corners per axis; total corners per axis
    int iters;
    double lam;
    int norm;               // 0 L2, 1 L1, 2 Huber (App. B iii)
    double huber_b;
    int stereo;             // 1: horizontal displacement only (App. I)
    int centre_map;
    double* patch;          // [N][4]: u, v, mean residual at u (channel 0), distance moved
    double* uinit;          // [N][2]
    int nc;                 // colour channels (App. B i); J0, J1 hold nc planes of W x H
    double* mdc;            // [N][nc] mean residual of every channel (nc > 1)
};

// Densification (Eq. 3) and the warped second frame for the refinement.
struct DensifyArgs {
    const double* J0;
    const double* J1;
    int W, H;
    const double* patch;
    int ps, st, nrx, nry, nx, ny;
    int raw_residual;
    double* U;              // [2][H][W]
    double* J1w;            // [nc][H][W], or null without refinement
    double* Z;              // [H][W] sum of the weights, or null (kept for the backward pass)
    int nc;                 // colour channels: J0, J1 hold nc planes
    const double* mdc;      // [N][nc] per-channel mean residuals (nc > 1)
};

// Part of one fixed-point iteration of the refinement: linearisation from
// J0 and the warped J1w, robust weights from the frozen increment dUf, then
// nhalf red-black half sweeps starting from dUin, written to dUout (and
// U + dU to Uout when non-null).
struct RefineArgs {
    const double* U;
    const double* J0;
    const double* J1w;
    const double* dUf;      // null = zero
    const double* dUin;     // null = zero
    double* dUout;
    double* Uout;
    double* tape;           // when non-null: state after half sweep m at tape + m*2*W*H (m >= 1)
    int tape_m0;            // half sweeps of this level done before this launch
    // linearisation of the level (Ix, Iy, Iz, Ixx, Ixy, Iyy, Ixz, Iyz and the
    // three normalisers: [11][H][W]); it depends on J0 and J1w only, so the
    // level's first launch writes it (lin_mode 1, core pixels) and later
    // launches read it for their pixels instead of recomputing (lin_mode 2)
    // With colour frames (lin_mode 3) the lin planes hold these 11 terms of
    // every channel ([nc][11][H][W]), written by k_colour_lin, and the tile
    // sums the data terms over the channels.
    double* lin;
    int lin_mode;           // 0 compute, 1 compute and store, 2 load, 3 colour (load every channel)
    int nc;
    int stereo;             // 1: relax du only, dv stays zero (App. I)
    int W, H;
    int nhalf;
    int tiles_x;
    double delta, gamma, alpha, omega, eps;
};

// Bilinear upscaling of the finest computed level to the output size.
struct UpsArgs {
    const double* U;
    int Ws, Hs;
    int W, H;
    double f;               // 2^theta_sf
    int centre_map;
    void* out;
    int out_f64;
    int rows;               // output rows per block
    const int* poison;      // non-null and set: a persistent wait of this plan gave up, the flow is written as NaN
};

// One pair at one level inside a persistent level launch.  Its work is a
// queue segment per phase: phase 0 = search blocks, phase 1 = densification
// blocks, phases 2.. = refinement steps (one tile each).
struct LevelPair {
    SearchArgs sa;
    DensifyArgs da;
    RefineArgs ra;          // the per-phase increment buffers come from RefPhase
    double* dU[3];
    int dens_bx;            // densification blocks per row
};

// Buffers of one refinement phase: indices into LevelPair::dU (-1 = zero).
struct RefPhase {
    int f, in, out;
    int nhalf;
    int last;               // 1: also write U + dU
    int m0;                 // half sweeps of the level before this phase (tape index)
};

// A persistent launch over the queue segments of every pair at one level,
// ordered phase-major; a task waits only for the previous phase of its own
// pair, which sits earlier in the queue, so the queue cannot deadlock.
struct LevelLaunch {
    const LevelPair* pairs;
    const RefPhase* rph;
    const int* start;       // [nph * npairs + 1] first task of each segment
    const int* task_seg;    // [ntasks] segment of each task (phase * npairs + pair)
    int* sync;              // [0] queue head, [1] wait-timeout flag, [2 + seg] finished tasks
    int* plan_err;          // every level launch of the plan sets this too when a wait gives up
    int fail_waits;         // failure-path testing: every wait of a later phase gives up at once
    int npairs, nph, ntasks;
    // the queue hands out runs of consecutive tasks of one segment: run r is
    // tasks run_start[r] .. run_start[r + 1] - 1, so one wait, one acquire and
    // one release cover the whole run
    const int* run_start;   // [nruns + 1]
    int nruns;
    int lin_cache;          // 1: a level's first refinement launch stores the linearisation, later ones load it
    // With one pair its arguments also travel in the launch itself: a
    // phase-major block then starts on its data at once, instead of after
    // a chain of dependent table reads (start, task_seg, pairs), each a
    // round trip to memory at the start of every launch.
    int one;                // 1: npairs == 1 and the fields below are set
    int dens_bx1;
    SearchArgs sa1;
    DensifyArgs da1;
};

// The refinement arguments of phase rp of pair P: the pair's, with the
// phase's increment buffers resolved.  A level's first refinement launch
// fills the linearisation cache, later ones read it; colour frames read the
// per-channel linearisation of k_colour_lin.  The kernels resolve it from
// the tables, the host for the arguments a single-pair launch carries.
__host__ __device__ inline RefineArgs dis_phase_args(const LevelPair& P, const RefPhase& rp, int lin_cache,
                                                     bool colour) {
    RefineArgs ra = P.ra;
    ra.dUf = rp.f < 0 ? nullptr : P.dU[rp.f];
    ra.dUin = rp.in < 0 ? nullptr : P.dU[rp.in];
    ra.dUout = P.dU[rp.out];
    ra.Uout = rp.last ? P.ra.Uout : nullptr;
    ra.nhalf = rp.nhalf;
    ra.tape_m0 = rp.m0;
    ra.lin_mode = colour ? 3 : (lin_cache ? (rp.m0 == 0 ? 1 : 2) : 0);
    return ra;
}

// A phase-major refinement launch: phase `phase` of every pair of L.
struct PhaseLaunch {
    LevelLaunch L;
    int phase;
    RefineArgs ra1;         // L.one: the pair's arguments with this phase's buffers resolved
};

// Pair-levels small enough for one workgroup's LDS (at most DIS_SMALL_PAIRS
// horizontal pixel pairs): densification and every refinement step of the
// level in one block, without tiles.  Block b handles pairs[list[b]].
#define DIS_SMALL_PAIRS 1024
#define DIS_SMALL_PX 2112      // LDS plane capacity (pixels) of that block
struct SmallLaunch {
    const LevelPair* pairs;
    const int* list;
    int n;
    int nouter;             // fixed-point steps of the level
    int nhalf;              // red-black half sweeps per step
    DensifyArgs da1;        // one pair (a single block): its arguments, read in place
    RefineArgs ra1;
};

// Forward-backward consistent densification (App. B ii): the two
// directions are pairs 0 (frame 0 -> 1) and 1 (1 -> 0) of one level launch.
// For direction d the other direction's patches are binned by the cell of
// their displaced corner floor(corner + u) (cells of ps x ps pixels, cell
// index offset by one so that corners down to -ps are kept); a pixel then
// looks at the 2 x 2 cells its covering patches can come from.
struct FbBins {
    int* count;             // [Wc * Hc], zero between uses (the scan clears it)
    int* start;             // [Wc * Hc + 1]
    int* cursor;            // [Wc * Hc]
    int* list;              // [N] patch indices grouped by cell
};
struct FbLaunch {
    LevelLaunch L;          // pairs 0 and 1 of this level
    FbBins bins[2];         // bins[d]: patches of direction 1 - d, displaced into frame d
    int Wc, Hc;
};
#define DIS_FB_MAXCAND 32     // covering candidates a pixel sorts in registers

// Table-driven multi-pair launches of the pyramid and the upscaling: entry
// j covers blocks start[j] .. start[j+1]-1.
struct PyrTab {
    const PyrArgs* tab;
    const int* start;
    const int* blk;         // [blocks]: the entry each block belongs to
    int n;
    int* zero;              // block 0 clears these ints (queue state of the level launches)
    int nzero;
};

struct UpsTab {
    const UpsArgs* tab;
    const int* start;
    const int* blk;         // [blocks]: the entry each block belongs to
    int n;
};

// Global-memory view of a device pointer.  Pointers that reach a kernel
// inside an argument structure copied to registers are generic, so their
// accesses compile to flat_* instructions, which also count against the LDS
// wait counter; through this view they are global_* ones (measured: 13.4 ->
// 12.9 us per refinement launch on the small scales).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* dis_global(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Workgroups are handed to the 8 XCDs round-robin (block b to XCD b mod 8),
// and each XCD has its own L2.  Blocks whose tiles share halo should sit on
// one XCD: this maps the blocks XCD x receives to the x-th contiguous run of
// n / 8 (or one more) tile indices.  A bijection on [0, n).
__device__ __forceinline__ int dis_xcd_tile(int b, int n) {
    const int x = b & 7, j = b >> 3, per = n >> 3, rem = n & 7;
    return x * per + (x < rem ? x : rem) + j;
}

// Order of the tiles of one pair inside its run of blocks: vertical bands
// bw tiles wide (bw ~ sqrt(n / 8), so that the n / 8 consecutive tiles one
// XCD receives form a near-square block), row-major inside a band, the last
// band narrower when bw does not divide tiles_x.  A bijection on [0, n) for
// n = tiles_x * tiles_y.
__device__ __forceinline__ int dis_band_tile(int q, int tiles_x, int n) {
    const int ty = n / tiles_x;
    int bw = 1;
    while ((bw + 1) * (bw + 1) * 8 <= n && bw + 1 <= tiles_x) ++bw;
    const int full = tiles_x / bw, span = bw * ty;
    int row, col;
    if (q < full * span) {
        const int band = q / span, r = q - band * span;
        row = r / bw;
        col = band * bw + (r - row * bw);
    } else {
        const int rw = tiles_x - full * bw, r = q - full * span;
        row = r / rw;
        col = full * bw + (r - row * rw);
    }
    return row * tiles_x + col;
}

// Kernel entry points, looked up by the host.
const void* dis_kernel_pyramid();
const void* dis_kernel_pyramid_tab();
const void* dis_kernel_upsample();
const void* dis_kernel_upsample_tab();
const void* dis_kernel_phase_search(int ps, int lpp);   // null when not compiled
const void* dis_kernel_phase_densify();
const void* dis_kernel_phase_refine(int tile);          // tile id, see dis_refine_tile
const void* dis_kernel_phase_refine_colour(int tile);   // colour frames (lin_mode 3)
const void* dis_kernel_phase_densify_colour();
const void* dis_kernel_small_level(int threads, bool one);   // SmallLaunch; 512 (<= 512 pairs) or 1024 threads
const void* dis_kernel_fb_count();                     // FbLaunch, grid (patch blocks, 2)
const void* dis_kernel_fb_scan();                      // FbLaunch, grid (1, 2), 1024 threads
const void* dis_kernel_fb_scatter();                   // FbLaunch, grid (patch blocks, 2)
const void* dis_kernel_fb_densify();                   // FbLaunch, grid (W/64, H/4, 2)
const void* dis_kernel_colour_lin();                   // LevelLaunch of one pair, grid of the densification
const void* dis_kernel_phase_search_colour(int ps);    // 3 channels; null when not compiled
int dis_colour_lanes(int ps);                          // its lanes per patch
const void* dis_kernel_level(int ps, int lpp);          // persistent level kernel, null when not compiled
// the row-owned search of grey frames with the L2 norm (64-thread blocks)
// and its persistent level kernel; null when no layout has lpp lanes
const void* dis_kernel_phase_search_rows(int ps, int lpp);
const void* dis_kernel_level_rows(int ps, int lpp, int tile);   // tile 0 or 1 (dis_level_tile)
// refinement core tile (width, height, threads per block) of a tile id;
// returns 0 for an unknown id
int dis_refine_tile(int tile, int* tw, int* th, int* nt);
// the lean tile id with the same core and threads as a tile id (itself when
// it is lean), or -1
int dis_refine_tile_lean(int tile);
#define DIS_NUM_TILES 13
