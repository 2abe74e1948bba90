// Handle layout and helpers shared by the host-side translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "dis.h"
#include "dis_internal.h"

// Device buffers of one pyramid level of one pair slot (float64, dense).
struct LevelBuf {
    double* J0;      // level image of frame 0 (0..255 scale; [nc][H][W] for colour frames)
    double* J1;      // level image of frame 1
    double* Ud;      // densified flow [2][H][W] (aliases U without refinement)
    double* U;       // flow after refinement [2][H][W]
    double* patch;   // [maxN][4]: u, v, mean residual, distance moved
    double* uinit;   // [maxN][2]
    double* mdc;     // [maxN][3] per-channel mean residuals (colour frames only)
    int maxN;
};

// Everything one frame pair needs; a handle owns max_batch of them.
struct SlotBuf {
    LevelBuf lv[DIS_MAXL];
    double* J1w;     // warped frame 1 of the level being refined ([nc][H][W])
    double* lin;     // [nc][11][H][W] linearisation of the level being refined
    double* dU[3];   // refinement increments (frozen / in / out rotation)
};

struct LevelGrid {
    int W, H, st, nrx, nry, nx, ny;
};

// One kernel launch with its argument block (kind: 0 internal, 1 reads the
// caller's frames, 2 writes the caller's flow).
struct Launch {
    const void* fn;
    dim3 grid, block;
    std::vector<char> arg;
    int kind;           // 3 reads the caller's flow gradient, 4 writes the frame gradients
    size_t shmem = 0;   // dynamic LDS bytes
    const char* name;   // kernel family, for profiling
    double bytes;       // algorithmic memory traffic of this launch
    double flops;       // algorithmic floating-point work of this launch
};

struct Seq {
    std::vector<Launch> items;
    void add(const void* fn, dim3 grid, dim3 block, const void* arg, size_t bytes, int kind,
             const char* name = "", double traffic = 0.0, double flops = 0.0);
};

struct ProfStat {
    int launches = 0;
    double ms = 0.0, bytes = 0.0, flops = 0.0;
};

struct ProfPending {
    hipEvent_t a, b;
    const char* name;
    int launches;           // consecutive launches of one family between the two events
    double bytes, flops;
};

struct PairInfo {
    int ss, sf;
};

// Device tables of a plan's persistent level launches (one allocation).
struct PlanTables {
    void* mem = nullptr;
    size_t bytes = 0;
    int* sync = nullptr;    // queue state of every level launch, cleared by the first pyramid launch
    int nsync = 0;
    std::vector<int> err_index;   // wait-timeout flag of each level launch inside sync
    int* plan_err = nullptr;      // inside sync: set by any level launch whose wait gave up (flows become NaN)
};

struct PairRef {
    SlotBuf* sb;
    int w, h;
    int ss;
};

struct Plan {
    Seq seq;
    PlanTables tabs;
    PairInfo info{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> nodes;
    const void* bound[3] = {nullptr, nullptr, nullptr};   // frames / flow the graph points at
};

// Device buffers of the backward pass (slot 0), allocated by dis_create when
// the handle keeps forward state for it.
struct BwdBuf {
    double* gJ0[DIS_MAXL];
    double* gJ1[DIS_MAXL];
    double* gU[DIS_MAXL];
    double* gP[DIS_MAXL];
    double* Z;
    double *gUd, *gJ1w, *gd, *gn, *acc, *coef, *gFacc;
    double* gq;      // [2][px] flow adjoint handed between the two densification passes
    double* tape;               // SOR states of one level, [half sweep][2][H][W]
    size_t tape_len;            // capacity in doubles
    size_t scratch_px;          // pixels of the largest processed level
};
struct BatchPlan;
void dis_batch_plan_free(BatchPlan* bp);
struct BwdPlan;
void dis_bwd_plan_free(BwdPlan* bp);

struct dis_handle {
    dis_params p;
    int max_w = 0, max_h = 0, max_batch = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    int st = 1;
    int top = 0;
    std::vector<void*> allocs;
    std::vector<SlotBuf> slots;
    std::string err;
    std::map<std::tuple<int, int, int>, Plan*> plans;
    std::map<std::vector<int>, BatchPlan*> bplans;
    int lpp[DIS_MAXL];
    int refine_tile = 7;
    int mode_phase = 1;     // 1: one launch per phase, 0: one persistent launch per level
    int small_levels = 0;   // single-launch refinement of scales of <= 256 (1) or <= 1024 (2) pixel pairs
    int bwd_reference = 0;  // backward: one launch per reverse half sweep instead of reverse tiles
    int no_lin_cache = 0;   // forward refinement recomputes the linearisation in every launch
    int fail_waits = 0;     // failure-path testing: persistent waits that would block give up at once
    int lean_big = 0;       // lean twin of the refinement tile on scales with at least two tiles per CU
    int n_cu = 256;
    // Static-scratch mode: device buffers are carved from [arena, arena +
    // arena_cap) instead of allocated; plans are single-pair and phase-major,
    // so no launch reads a device table.
    char* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    // most recent plain forward call (debug and backward)
    bool have_last = false;
    int last_w = 0, last_h = 0, last_ss = 0, last_sf = 0, last_pitch = 0;
    const void* last_I0 = nullptr;
    const void* last_I1 = nullptr;
    const PlanTables* last_tabs = nullptr;
    // the most recent forward call, replayed by the autotuner
    int last_call = 0;          // 0 none, 1 plain, 2 batched
    void* last_flow = nullptr;
    std::vector<const void*> last_batch, last_batch_I1;
    std::vector<void*> last_batch_flow;
    std::vector<int> last_batch_w, last_batch_h, last_batch_pitch;
    double tuned_ms = 0.0;
    // backward pass
    BwdBuf bwd{};
    std::map<std::tuple<int, int>, BwdPlan*> bwplans;
    // per-kernel event timing (dis_profile_enable)
    bool profiling = false;
    std::vector<ProfPending> prof_pending;
    std::vector<hipEvent_t> prof_free;
    std::map<std::string, ProfStat> prof;
};

int dis_stride(const dis_params* p);
int dis_validate_params(const dis_params* p);
int dis_top_level(const dis_params* p, int max_w, int max_h);
int dis_alloc_slot(dis_handle* h, SlotBuf& sb);
// image channels of a parameter block: 3 with DIS_FLAG_COLOUR, else 1
inline int dis_channels(const dis_params* p) { return (p->flags & DIS_FLAG_COLOUR) ? 3 : 1; }
int dis_coarsest(const dis_params* p, int w, int h);
void dis_grid(int n, int ps, int st, int* nr, int* ntot);
int dis_pick_lpp(const dis_handle* h, int s);
bool dis_search_rows_path(const dis_params* p);
bool dis_search_has_lanes(const dis_params* p, int lpp);
int dis_build_pair(dis_handle* h, SlotBuf& sb, int w, int hgt, int pitch, const void* I0, const void* I1,
                   void* flow, Seq& seq, PairInfo* info, PlanTables& tabs);
// Options of dis_build_levels for the backward pass's recomputation.
struct LevelOpts {
    int only_level = -1;        // build only this scale
    double* tape = nullptr;     // record every SOR half sweep's state
    double* Z = nullptr;        // keep the densification weight sums
    int skip_search = 0;        // the patch records are kept: recompute from densification on
    int force_phase = 0;        // one launch per phase whatever the tuned launch mode
};

int dis_alloc_backward(dis_handle* h);
// A single-pair forward of this handle records its finest scale's weight sums,
// SOR tape, warped frame and linearisation in the adjoint's buffers, and the
// adjoint starts from them instead of recomputing that scale.
bool dis_forward_keeps_finest(const dis_handle* h);
int dis_dalloc(dis_handle* h, void** ptr, size_t bytes);
int dis_build_graph_seq(dis_handle* h, Seq& seq, hipGraph_t* graph, hipGraphExec_t* exec,
                        std::vector<hipGraphNode_t>* nodes);
int dis_update_graph_seq(dis_handle* h, Seq& seq, hipGraphExec_t exec, const std::vector<hipGraphNode_t>& nodes);
int dis_level_grid(const dis_handle* h, int W, int H, LevelGrid* g);   // patch grid of a W x H level; returns N
int dis_build_levels(dis_handle* h, const std::vector<PairRef>& pairs, Seq& seq, PlanTables& tabs,
                     const LevelOpts* opt);
void dis_refine_phases(const dis_params& p, int s, std::vector<RefPhase>& out);
int dis_add_pyramid(dis_handle* h, SlotBuf& sb, int w, int hgt, int pitch, int ss, const void* I0, const void* I1,
                    Seq& seq);
void dis_add_upsample(dis_handle* h, SlotBuf& sb, int w, int hgt, void* flow, const int* poison, Seq& seq);
int dis_fail(dis_handle* h, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int dis_launch_eager(dis_handle* h, Seq& seq);
