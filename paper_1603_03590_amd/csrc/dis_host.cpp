// Host side of the Dense Inverse Search library: parameter validation, the
// per-handle device arena, launch sequences per frame size, HIP graph replay.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "dis.h"
#include "dis_internal.h"
#include "dis_host.h"

// ------------------------------------------------------------------ helpers

static thread_local std::string g_null_err;

static int fail(dis_handle* h, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
static int fail(dis_handle* h, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf; else g_null_err = buf;
    return code;
}

int dis_fail(dis_handle* h, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf; else g_null_err = buf;
    return code;
}

#define HIPCHK(h, call)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((h), DIS_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));       \
    } while (0)

static bool is_supported_ps(int ps) { return ps >= 4 && ps <= 16 && ps % 2 == 0; }

int dis_stride(const dis_params* p) {
    const double s = std::floor((double)p->patch_size * (1.0 - p->overlap));
    return s < 1.0 ? 1 : (int)s;
}

int dis_coarsest(const dis_params* p, int w, int h) {
    int s;
    if (p->coarsest_scale >= 0) {
        s = p->coarsest_scale;
    } else {
        // smallest s with 2^s >= 2 w / (8 ps)   (Sec. 3.1 rule, f = 8)
        s = 0;
        while ((double)(1LL << s) * 8.0 * p->patch_size < 2.0 * w) ++s;
    }
    if (s > DIS_MAXL - 1) s = DIS_MAXL - 1;
    while (s > 0 && ((w >> s) < p->patch_size || (h >> s) < p->patch_size)) --s;
    return s;
}

void dis_grid(int n, int ps, int st, int* nr, int* ntot) {
    *nr = (n - ps) / st + 1;
    *ntot = *nr + (((n - ps) % st) != 0 ? 1 : 0);
}

static int validate_params(const dis_params* p);
int dis_validate_params(const dis_params* p) { return validate_params(p); }

static int validate_params(const dis_params* p) {
    if (!p) return fail(nullptr, DIS_EINVAL, "params is NULL");
    if (!is_supported_ps(p->patch_size))
        return fail(nullptr, DIS_EINVAL, "patch_size %d unsupported (even, 4..16)", p->patch_size);
    if (!(p->overlap >= 0.0 && p->overlap < 1.0))
        return fail(nullptr, DIS_EINVAL, "overlap %g outside [0, 1)", p->overlap);
    if (p->coarsest_scale < -1 || p->coarsest_scale >= DIS_MAXL)
        return fail(nullptr, DIS_EINVAL, "coarsest_scale %d outside [-1, %d]", p->coarsest_scale, DIS_MAXL - 1);
    if (p->finest_scale < 0 || p->finest_scale >= DIS_MAXL)
        return fail(nullptr, DIS_EINVAL, "finest_scale %d outside [0, %d]", p->finest_scale, DIS_MAXL - 1);
    if (p->coarsest_scale >= 0 && p->finest_scale > p->coarsest_scale)
        return fail(nullptr, DIS_EINVAL, "finest_scale %d above coarsest_scale %d", p->finest_scale,
                    p->coarsest_scale);
    if (p->gn_iters < 0 || p->gn_iters > 100000)
        return fail(nullptr, DIS_EINVAL, "gn_iters %d outside [0, 100000]", p->gn_iters);
    if (p->refine) {
        if (p->var_outer < -1 || p->var_outer > 1000)
            return fail(nullptr, DIS_EINVAL, "var_outer %d outside [-1, 1000]", p->var_outer);
        if (p->var_inner < 1 || p->var_inner > 100000)
            return fail(nullptr, DIS_EINVAL, "var_inner %d outside [1, 100000]", p->var_inner);
        if (!(p->sor_omega > 0.0 && p->sor_omega < 2.0))
            return fail(nullptr, DIS_EINVAL, "sor_omega %g outside (0, 2)", p->sor_omega);
        if (!(p->w_intensity >= 0.0) || !(p->w_gradient >= 0.0) || !(p->w_smooth >= 0.0))
            return fail(nullptr, DIS_EINVAL, "refinement weights must be >= 0");
    }
    if (p->refine != 0 && p->refine != 1) return fail(nullptr, DIS_EINVAL, "refine must be 0 or 1");
    if (p->norm < DIS_NORM_L2 || p->norm > DIS_NORM_HUBER) return fail(nullptr, DIS_EINVAL, "norm %d unknown", p->norm);
    if (!(p->huber_b > 0.0)) return fail(nullptr, DIS_EINVAL, "huber_b %g must be > 0", p->huber_b);
    const uint32_t known = DIS_FLAG_KEEP_FOR_BACKWARD | DIS_FLAG_NO_GRAPH | DIS_FLAG_PIXEL_CENTRE |
                           DIS_FLAG_RAW_RESIDUAL | DIS_FLAG_IO_F64 | DIS_FLAG_STEREO |
                           DIS_FLAG_FB_CONSISTENCY | DIS_FLAG_COLOUR;
    if (p->flags & ~known) return fail(nullptr, DIS_EINVAL, "unknown flag bits 0x%x", p->flags & ~known);
    if (p->flags & DIS_FLAG_COLOUR) {
        if (p->flags & DIS_FLAG_FB_CONSISTENCY)
            return fail(nullptr, DIS_EINVAL, "colour frames and forward-backward consistency do not combine");
        if (!dis_kernel_phase_search_colour(p->patch_size))
            return fail(nullptr, DIS_EINVAL, "colour frames support patch sizes 4..12, not %d", p->patch_size);
    }
    return DIS_OK;
}

// ------------------------------------------------------------------ presets

extern "C" int dis_default_params(int preset, dis_params* out) {
    if (!out) return fail(nullptr, DIS_EINVAL, "out is NULL");
    dis_params p;
    std::memset(&p, 0, sizeof p);
    p.coarsest_scale = 5;
    p.var_outer = -1;
    p.var_inner = 5;
    p.w_intensity = 5.0;
    p.w_gradient = 10.0;
    p.w_smooth = 10.0;
    p.sor_omega = 1.6;
    p.refine = 1;
    p.flags = 0;
    p.norm = DIS_NORM_L2;
    p.huber_b = 1.0;
    switch (preset) {
        case 1: p.finest_scale = 3; p.gn_iters = 16; p.patch_size = 8; p.overlap = 0.3; p.refine = 0; break;
        case 2: p.finest_scale = 3; p.gn_iters = 12; p.patch_size = 8; p.overlap = 0.4; break;
        case 3: p.finest_scale = 1; p.gn_iters = 16; p.patch_size = 12; p.overlap = 0.75; break;
        case 4: p.finest_scale = 0; p.gn_iters = 256; p.patch_size = 12; p.overlap = 0.75; break;
        case 101: p.patch_size = 8; p.overlap = 0.3; p.coarsest_scale = 2; p.finest_scale = 0;
                  p.gn_iters = 8; p.var_outer = 1; break;
        case 102: p.patch_size = 8; p.overlap = 0.3; p.finest_scale = 3; p.gn_iters = 12; break;
        case 103: p.patch_size = 8; p.overlap = 0.5; p.finest_scale = 3; p.gn_iters = 16; break;
        case 104: p.patch_size = 12; p.overlap = 0.75; p.coarsest_scale = 4; p.finest_scale = 0;
                  p.gn_iters = 128; p.var_outer = 5; break;
        case 105: p.patch_size = 8; p.overlap = 0.5; p.coarsest_scale = 3; p.finest_scale = 0;
                  p.gn_iters = 16; p.var_outer = 3; break;
        case 106: p.patch_size = 8; p.overlap = 0.5; p.coarsest_scale = -1; p.finest_scale = 3;
                  p.gn_iters = 16; break;
        default: return fail(nullptr, DIS_EINVAL, "unknown preset %d", preset);
    }
    *out = p;
    return DIS_OK;
}

// ------------------------------------------------------------------- arena

int dis_dalloc(dis_handle* h, void** ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) return DIS_OK;
    if (h->arena) {
        const size_t off = (h->arena_used + 255) & ~(size_t)255;
        if (off > h->arena_cap || bytes > h->arena_cap - off)
            return fail(h, DIS_ESIZE, "the frame needs more than the %zu bytes of static scratch", h->arena_cap);
        *ptr = h->arena + off;
        h->arena_used = off + bytes;
        return DIS_OK;
    }
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
            return fail(h, DIS_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return fail(h, DIS_EHIP, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    h->allocs.push_back(*ptr);
    return DIS_OK;
}

#define DALLOC(h, ptr, bytes)                                      \
    do {                                                           \
        int r_ = dis_dalloc((h), (void**)&(ptr), (bytes));         \
        if (r_ != DIS_OK) return r_;                               \
    } while (0)

int dis_alloc_slot(dis_handle* h, SlotBuf& sb) {
    const dis_params& p = h->p;
    const int W = h->max_w, H = h->max_h, ps = p.patch_size, st = h->st;
    const int nc = dis_channels(&p);
    std::memset(&sb, 0, sizeof sb);
    for (int s = 0; s <= h->top; ++s) {
        LevelBuf& L = sb.lv[s];
        const int ws = W >> s, hs = H >> s;
        const size_t px = (size_t)ws * hs;
        // level images: the processed levels, and every fifth level (a later
        // pyramid pass starts from it)
        if (s >= p.finest_scale || (s > 0 && s % 5 == 0)) {
            DALLOC(h, L.J0, nc * px * sizeof(double));
            DALLOC(h, L.J1, nc * px * sizeof(double));
        }
        if (s >= p.finest_scale && ws >= ps && hs >= ps) {
            const int nx = (ws - ps) / st + 2, ny = (hs - ps) / st + 2;
            L.maxN = nx * ny;
            DALLOC(h, L.patch, (size_t)L.maxN * 4 * sizeof(double));
            DALLOC(h, L.uinit, (size_t)L.maxN * 2 * sizeof(double));
            if (nc > 1) DALLOC(h, L.mdc, (size_t)L.maxN * nc * sizeof(double));
            DALLOC(h, L.U, 2 * px * sizeof(double));
            if (p.refine) DALLOC(h, L.Ud, 2 * px * sizeof(double));
            else L.Ud = L.U;
        }
    }
    const int sf = p.finest_scale;
    const size_t pf = (size_t)(W >> sf) * (H >> sf);
    if (p.refine) {
        DALLOC(h, sb.J1w, nc * pf * sizeof(double));
        // without the linearisation cache only colour frames use this buffer
        if (!h->no_lin_cache || nc > 1) DALLOC(h, sb.lin, 11 * nc * pf * sizeof(double));
        for (int i = 0; i < 3; ++i) DALLOC(h, sb.dU[i], 2 * pf * sizeof(double));
    }
    return DIS_OK;
}

// Deepest pyramid level whose frames still hold a patch, for max_w x max_h.
int dis_top_level(const dis_params* p, int max_w, int max_h) {
    int top = 0;
    while (top + 1 < DIS_MAXL && (max_w >> (top + 1)) >= p->patch_size && (max_h >> (top + 1)) >= p->patch_size) ++top;
    return top;
}

extern "C" int dis_create(const dis_params* p, int max_w, int max_h, int max_batch, void* stream,
                          dis_handle** out) {
    if (!out) return fail(nullptr, DIS_EINVAL, "out is NULL");
    *out = nullptr;
    int r = validate_params(p);
    if (r != DIS_OK) return r;
    if (max_batch < 1 || max_batch > 4096) return fail(nullptr, DIS_EINVAL, "max_batch %d outside [1, 4096]", max_batch);
    if (max_w < 1 || max_h < 1 || max_w > 65536 || max_h > 65536)
        return fail(nullptr, DIS_EINVAL, "max size %dx%d invalid", max_w, max_h);
    if ((max_w >> p->finest_scale) < p->patch_size || (max_h >> p->finest_scale) < p->patch_size)
        return fail(nullptr, DIS_ESIZE, "%dx%d at scale %d is smaller than the %d px patch", max_w, max_h,
                    p->finest_scale, p->patch_size);
    dis_handle* h = new dis_handle();
    h->p = *p;
    h->max_w = max_w;
    h->max_h = max_h;
    h->max_batch = max_batch;
    h->stream = (hipStream_t)stream;
    h->st = dis_stride(p);
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(nullptr, DIS_EHIP, "hipGetDevice failed");
    }
    {
        hipDeviceProp_t prop;
        h->n_cu = hipGetDeviceProperties(&prop, h->device) == hipSuccess ? prop.multiProcessorCount : 256;
        if (h->n_cu < 1) h->n_cu = 256;
    }
    h->top = dis_top_level(p, max_w, max_h);
    for (int s = 0; s < DIS_MAXL; ++s) h->lpp[s] = 0;
    h->refine_tile = 7;   // 8x8 cores, 512 threads: the fastest on small scales
    const bool fb = (p->flags & DIS_FLAG_FB_CONSISTENCY) != 0;
    const int nslots = fb ? std::max(max_batch, 2) : max_batch;
    h->slots.resize(nslots);
    for (int i = 0; i < nslots; ++i) {
        r = dis_alloc_slot(h, h->slots[i]);
        if (r != DIS_OK) {
            g_null_err = h->err;
            dis_destroy(h);
            return r;
        }
    }
    if (fb) {
        // the backward direction (slot 1) reads the same pyramid, frames swapped
        for (int s = 0; s < DIS_MAXL; ++s) {
            h->slots[1].lv[s].J0 = h->slots[0].lv[s].J1;
            h->slots[1].lv[s].J1 = h->slots[0].lv[s].J0;
        }
    }
    if (p->flags & DIS_FLAG_KEEP_FOR_BACKWARD) {
        r = dis_alloc_backward(h);
        if (r != DIS_OK) {
            g_null_err = h->err;
            dis_destroy(h);
            return r;
        }
    }
    *out = h;
    return DIS_OK;
}

extern "C" void dis_destroy(dis_handle* h) {
    if (!h) return;
    hipStreamSynchronize(h->stream);
    for (auto& kv : h->plans) {
        Plan* pl = kv.second;
        if (pl->exec) hipGraphExecDestroy(pl->exec);
        if (pl->graph) hipGraphDestroy(pl->graph);
        if (pl->tabs.mem) hipFree(pl->tabs.mem);
        delete pl;
    }
    for (auto& kv : h->bplans) {
        BatchPlan* bp = kv.second;
        dis_batch_plan_free(bp);
    }
    for (auto& kv : h->bwplans) dis_bwd_plan_free(kv.second);
    for (ProfPending& pp : h->prof_pending) { hipEventDestroy(pp.a); hipEventDestroy(pp.b); }
    for (hipEvent_t e : h->prof_free) hipEventDestroy(e);
    for (void* ptr : h->allocs) hipFree(ptr);
    delete h;
}

extern "C" const char* dis_last_error(const dis_handle* h) {
    return h ? h->err.c_str() : g_null_err.c_str();
}

static void drop_plans(dis_handle* h) {
    hipStreamSynchronize(h->stream);
    for (auto& kv : h->plans) {
        Plan* pl = kv.second;
        if (pl->exec) hipGraphExecDestroy(pl->exec);
        if (pl->graph) hipGraphDestroy(pl->graph);
        if (pl->tabs.mem) hipFree(pl->tabs.mem);
        delete pl;
    }
    h->plans.clear();
    for (auto& kv : h->bplans) dis_batch_plan_free(kv.second);
    h->bplans.clear();
    for (auto& kv : h->bwplans) dis_bwd_plan_free(kv.second);
    h->bwplans.clear();
}

extern "C" int dis_set_tunables(dis_handle* h, const int* lanes_per_patch, int refine_tile, int launch_mode) {
    if (!h) return fail(nullptr, DIS_EINVAL, "handle is NULL");
    int tw, th;
    if (!dis_refine_tile(refine_tile, &tw, &th, nullptr))
        return fail(h, DIS_EINVAL, "unknown refinement tile %d", refine_tile);
    if (launch_mode < 0 || launch_mode > 127) return fail(h, DIS_EINVAL, "launch mode %d outside 0..127", launch_mode);
    if (lanes_per_patch)
        for (int s = 0; s < DIS_MAXL; ++s) {
            const int l = lanes_per_patch[s];
            if (l != 0 && !dis_kernel_phase_search(h->p.patch_size, l) &&
                !dis_kernel_phase_search_rows(h->p.patch_size, l))
                return fail(h, DIS_EINVAL, "no search kernel for patch %d with %d lanes", h->p.patch_size, l);
        }
    drop_plans(h);
    for (int s = 0; s < DIS_MAXL; ++s) h->lpp[s] = lanes_per_patch ? lanes_per_patch[s] : 0;
    h->refine_tile = refine_tile;
    h->mode_phase = launch_mode & 1;
    h->small_levels = (launch_mode & 2) ? ((launch_mode & 16) ? 2 : 1) : 0;
    h->bwd_reference = (launch_mode & 4) ? 1 : 0;
    h->no_lin_cache = (launch_mode & 8) ? 1 : 0;
    h->fail_waits = (launch_mode & 32) ? 1 : 0;
    h->lean_big = (launch_mode & 64) ? 1 : 0;
    return DIS_OK;
}

extern "C" int dis_get_tunables(const dis_handle* h, int* lanes_per_patch, int* refine_tile, int* launch_mode) {
    if (!h) return fail(nullptr, DIS_EINVAL, "handle is NULL");
    if (lanes_per_patch)
        for (int s = 0; s < DIS_MAXL; ++s) lanes_per_patch[s] = h->lpp[s];
    if (refine_tile) *refine_tile = h->refine_tile;
    if (launch_mode)
        *launch_mode = h->mode_phase | (h->small_levels ? 2 : 0) | (h->bwd_reference ? 4 : 0) | (h->no_lin_cache ? 8 : 0) |
                       (h->small_levels == 2 ? 16 : 0) | (h->fail_waits ? 32 : 0) | (h->lean_big ? 64 : 0);
    return DIS_OK;
}

extern "C" int dis_set_stream(dis_handle* h, void* stream) {
    if (!h) return fail(nullptr, DIS_EINVAL, "handle is NULL");
    h->stream = (hipStream_t)stream;
    return DIS_OK;
}

// ------------------------------------------------------------ launch lists

void Seq::add(const void* fn, dim3 grid, dim3 block, const void* arg, size_t bytes, int kind, const char* name,
              double traffic, double flops) {
    Launch L;
    L.fn = fn;
    L.grid = grid;
    L.block = block;
    L.arg.assign((const char*)arg, (const char*)arg + bytes);
    L.kind = kind;
    L.name = name;
    L.bytes = traffic;
    L.flops = flops;
    items.push_back(std::move(L));
}

// Grey frames with the L2 norm take the row-owned search where a layout is
// compiled for the patch size; colour frames and the robust norms the
// per-pixel one.
bool dis_search_rows_path(const dis_params* p) {
    if (dis_channels(p) != 1 || p->norm != DIS_NORM_L2) return false;
    for (int l = 1; l <= 16; l <<= 1)
        if (dis_kernel_phase_search_rows(p->patch_size, l)) return true;
    return false;
}

// Is `lpp` a lanes-per-patch count of the search this parameter block uses?
bool dis_search_has_lanes(const dis_params* p, int lpp) {
    return dis_search_rows_path(p) ? dis_kernel_phase_search_rows(p->patch_size, lpp) != nullptr
                                   : dis_kernel_phase_search(p->patch_size, lpp) != nullptr;
}

int dis_pick_lpp(const dis_handle* h, int s) {
    const int ps = h->p.patch_size;
    // a requested count the search was not compiled for falls back to the default
    if (h->lpp[s] && dis_search_has_lanes(&h->p, h->lpp[s])) return h->lpp[s];
    // the most lanes compiled for the patch size: the shortest dependent chain
    // per patch (the autotuner tries the others)
    if (dis_search_rows_path(&h->p)) {
        for (int l = 16; l >= 1; l >>= 1)
            if (dis_kernel_phase_search_rows(ps, l)) return l;
    }
    for (int l = 64; l > 16; l >>= 1)
        if (dis_kernel_phase_search(ps, l)) return l;
    return 16;
}

int dis_level_grid(const dis_handle* h, int W, int H, LevelGrid* g) {
    const int ps = h->p.patch_size;
    g->W = W;
    g->H = H;
    g->st = h->st;
    dis_grid(W, ps, h->st, &g->nrx, &g->nx);
    dis_grid(H, ps, h->st, &g->nry, &g->ny);
    return g->nx * g->ny;
}

// ------------------------------------------------------- cost models
// Algorithmic traffic (bytes every launch must move) and floating-point work
// per kernel family, from the sizes of the arrays each one reads and writes.

static double search_bytes(double px, double pxn, double N) { return 16.0 * px + 16.0 * pxn + 48.0 * N; }
static double search_flops(double N, double P, int iters) {
    // Sobel + Hessian setup 24/px, 15/px and 20 per Gauss-Newton iteration,
    // 10/px for the final residual
    return N * (24.0 * P + iters * (15.0 * P + 20.0) + 10.0 * P);
}
static double densify_bytes(double px, double N, bool refine) { return 32.0 * px + 32.0 * N + (refine ? 8.0 * px : 0.0); }
static double densify_flops(double px, double cover, bool refine) { return px * (18.0 * cover + 2.0 + (refine ? 9.0 : 0.0)); }
static double refine_bytes(double px, bool f, bool in, bool last) {
    // J0, J1w, U, frozen and starting increments in; increment (and flow) out
    return px * (16.0 + 16.0 + (f ? 16.0 : 0.0) + (in ? 16.0 : 0.0) + 16.0 + (last ? 16.0 : 0.0));
}
static double refine_flops(double px, int nhalf) {
    // 155 per pixel for linearisation, weights and coefficients, 24 per pixel
    // update (half of the pixels each half sweep)
    return px * (155.0 + 12.0 * nhalf);
}

// ------------------------------------------------------- launch sequences

// Pyramid pass(es) of one pair: levels a+1 .. a+5 from level a.
int dis_add_pyramid(dis_handle* h, SlotBuf& sb, int w, int hgt, int pitch, int ss, const void* I0,
                       const void* I1, Seq& seq) {
    const dis_params& p = h->p;
    const int sf = p.finest_scale;
    const bool f64io = (p.flags & DIS_FLAG_IO_F64) != 0;
    const int nc = dis_channels(&p);
    for (int a = 0; a < ss || (a == 0 && ss == 0); a += 5) {
        PyrArgs pa;
        std::memset(&pa, 0, sizeof pa);
        const int w0 = w >> a, h0 = hgt >> a;
        pa.nc = nc;
        pa.src_cstride = a == 0 ? (long long)hgt * pitch : (long long)w0 * h0;
        pa.a = a;
        pa.nlev = std::min(5, ss - a);
        pa.w0 = w0;
        pa.h0 = h0;
        if (a == 0) {
            pa.src[0] = I0;
            pa.src[1] = I1;
            pa.src_kind = f64io ? 2 : 1;
            pa.src_pitch = pitch;
            pa.scale = 255.0;
            if (sf == 0) { pa.lvl0[0] = sb.lv[0].J0; pa.lvl0[1] = sb.lv[0].J1; }
        } else {
            pa.src[0] = sb.lv[a].J0;
            pa.src[1] = sb.lv[a].J1;
            pa.src_kind = 0;
            pa.src_pitch = w0;
            pa.scale = 1.0;
        }
        for (int k = 1; k <= pa.nlev; ++k) {
            const int s = a + k;
            pa.ws[k] = w >> s;
            pa.hs[k] = hgt >> s;
            // keep the levels that are processed, and the start of the next pass
            if (s >= sf || (s == a + 5 && s < ss)) { pa.dst[0][k] = sb.lv[s].J0; pa.dst[1][k] = sb.lv[s].J1; }
        }
        pa.tiles_x = (w0 + 255) / 256;
        const int tiles = dis_pyramid_tiles(pa);
        // traffic: both frames of level a in, every kept level out (float64)
        double by = 2.0 * (double)w0 * h0 * (a == 0 ? (f64io ? 8 : 4) : 8), fl = a == 0 ? 2.0 * w0 * h0 : 0.0;
        if (pa.lvl0[0]) by += 16.0 * w0 * h0;
        for (int k = 1; k <= pa.nlev; ++k) {
            const double px = (double)pa.ws[k] * pa.hs[k];
            fl += 2.0 * 4.0 * px;
            if (pa.dst[0][k]) by += 16.0 * px;
        }
        seq.add(dis_kernel_pyramid(), dim3(tiles, 2 * nc), dim3(DIS_PYR_THREADS), &pa, sizeof pa, a == 0 ? 1 : 0, "pyramid",
                nc * by, nc * fl);
        if (ss == 0) break;
    }
    return DIS_OK;
}

void dis_add_upsample(dis_handle* h, SlotBuf& sb, int w, int hgt, void* flow, const int* poison, Seq& seq) {
    const dis_params& p = h->p;
    const int sf = p.finest_scale;
    const bool f64io = (p.flags & DIS_FLAG_IO_F64) != 0;
    UpsArgs ua;
    std::memset(&ua, 0, sizeof ua);
    ua.U = sb.lv[sf].U;
    ua.Ws = w >> sf;
    ua.Hs = hgt >> sf;
    ua.W = w;
    ua.H = hgt;
    ua.f = (double)(1 << sf);
    ua.centre_map = (p.flags & DIS_FLAG_PIXEL_CENTRE) ? 1 : 0;
    ua.out = flow;
    ua.out_f64 = f64io ? 1 : 0;
    ua.poison = poison;
    ua.rows = dis_upsample_rows(w, hgt);
    seq.add(dis_kernel_upsample(), dim3((w + 255) / 256, dis_upsample_blocks_y(w, hgt)), dim3(256), &ua, sizeof ua, 2, "upsample",
            16.0 * ua.Ws * ua.Hs + (f64io ? 16.0 : 8.0) * w * hgt, 20.0 * w * hgt);
}

// Refinement phases of one level: theta_vo fixed-point steps, each split
// into launches of at most DIS_KMAX half sweeps; three increment buffers
// rotate so that a phase never writes what it reads.
void dis_refine_phases(const dis_params& p, int s, std::vector<RefPhase>& out) {
    out.clear();
    const int nouter = p.var_outer < 0 ? s + 1 : p.var_outer;
    if (nouter == 0) {
        out.push_back(RefPhase{-1, -1, 0, 0, 1, 0});
        return;
    }
    int cur = -1, m = 0;
    for (int k = 0; k < nouter; ++k) {
        const int frozen = cur;
        int in = cur;
        int left = 2 * p.var_inner;
        while (left > 0) {
            const int nh = std::min(left, DIS_KMAX);
            left -= nh;
            int ob = 0;
            while (ob == frozen || ob == in) ++ob;
            out.push_back(RefPhase{frozen, in, ob, nh, (k == nouter - 1 && left == 0) ? 1 : 0, m});
            m += nh;
            in = ob;
        }
        cur = in;
    }
}

bool dis_forward_keeps_finest(const dis_handle* h) {
    const dis_params& p = h->p;
    return (p.flags & DIS_FLAG_KEEP_FOR_BACKWARD) && p.refine && !(p.flags & DIS_FLAG_FB_CONSISTENCY) &&
           dis_channels(&p) == 1 && h->bwd.tape != nullptr && h->bwd.Z != nullptr;
}

// Search, densification and refinement of every pair at every level.
// The per-level work is laid out as queue segments (phase-major, then pair)
// in device tables; launch mode 0 runs each level as one persistent k_level
// launch over that queue, mode 1 as one launch per phase covering every
// pair.  Both give the same bits.
int dis_build_levels(dis_handle* h, const std::vector<PairRef>& pairs, Seq& seq, PlanTables& tabs,
                     const LevelOpts* opt) {
    const dis_params& p = h->p;
    const int ps = p.patch_size, sf = p.finest_scale;
    const int cmap = (p.flags & DIS_FLAG_PIXEL_CENTRE) ? 1 : 0;
    int top = sf;
    for (const PairRef& r : pairs) top = std::max(top, r.ss);
    const bool fbm = (p.flags & DIS_FLAG_FB_CONSISTENCY) && !opt && pairs.size() == 2;
    const int nc = dis_channels(&p);
    const bool keep_tape = !opt && pairs.size() == 1 && dis_forward_keeps_finest(h);
    // colour frames and the merged densification run phase-major only
    const int mode = ((opt && opt->force_phase) || fbm || nc > 1 || h->arena) ? 1 : h->mode_phase;
    // static-scratch plans carry every argument in the launches themselves
    const bool no_tables = h->arena != nullptr;
    if (no_tables && (pairs.size() != 1 || opt))
        return fail(h, DIS_EINVAL, "internal: a static-scratch plan holds one pair and no recomputation");
    const int tile_id = mode ? h->refine_tile : dis_level_tile(h->refine_tile, nc == 1 && dis_search_rows_path(&p));
    int tw = 32, th = 16, nt = 256;
    dis_refine_tile(tile_id, &tw, &th, &nt);

    struct LevelHost {
        std::vector<LevelPair> lp;
        std::vector<RefPhase> rph;
        std::vector<int> small;     // pairs refined by one single-workgroup launch
        std::vector<char> is_small;
        int s;
        int lpp;
        int nph;
        double by[2], fl[2], sby, sfl;
    };
    std::vector<LevelHost> levels;
    for (int s = top; s >= sf; --s) {
        if (opt && opt->only_level >= 0 && s != opt->only_level) continue;
        LevelHost LH;
        LH.s = s;
        LH.sby = LH.sfl = 0.0;
        dis_refine_phases(p, s, LH.rph);
        if (!p.refine) LH.rph.clear();
        LH.nph = 2 + (int)LH.rph.size();
        LH.lpp = nc > 1 ? dis_colour_lanes(ps) : dis_pick_lpp(h, s);
        LH.by[0] = LH.by[1] = LH.fl[0] = LH.fl[1] = 0.0;
        for (const PairRef& r : pairs) {
            if (r.ss < s) continue;
            SlotBuf& sb = *r.sb;
            LevelBuf& L = sb.lv[s];
            LevelGrid g;
            const int N = dis_level_grid(h, r.w >> s, r.h >> s, &g);
            if (N > L.maxN) return fail(h, DIS_ESIZE, "internal: %d patches exceed capacity %d", N, L.maxN);
            const int W = g.W, Hh = g.H;
            LevelPair P;
            std::memset(&P, 0, sizeof P);
            SearchArgs& sa = P.sa;
            sa.J0 = L.J0; sa.J1 = L.J1; sa.W = W; sa.H = Hh;
            if (s < r.ss) { sa.Un = sb.lv[s + 1].U; sa.Wn = r.w >> (s + 1); sa.Hn = r.h >> (s + 1); }
            sa.st = g.st; sa.nrx = g.nrx; sa.nry = g.nry; sa.nx = g.nx; sa.ny = g.ny;
            sa.iters = p.gn_iters;
            sa.lam = 1e-3;
            sa.norm = p.norm;
            sa.huber_b = p.huber_b;
            sa.stereo = (p.flags & DIS_FLAG_STEREO) ? 1 : 0;
            sa.centre_map = cmap;
            sa.patch = L.patch;
            sa.uinit = L.uinit;
            sa.nc = nc;
            sa.mdc = L.mdc;
            DensifyArgs& da = P.da;
            da.J0 = L.J0; da.J1 = L.J1; da.W = W; da.H = Hh;
            da.patch = L.patch;
            da.ps = ps; da.st = g.st; da.nrx = g.nrx; da.nry = g.nry; da.nx = g.nx; da.ny = g.ny;
            da.raw_residual = (p.flags & DIS_FLAG_RAW_RESIDUAL) ? 1 : 0;
            da.U = L.Ud;
            da.J1w = p.refine ? sb.J1w : nullptr;
            // a forward kept for the adjoint records the finest scale's SOR
            // tape and weight sums as it goes, so the adjoint starts there
            // without recomputing that scale (the buffers hold one scale)
            const bool record = keep_tape && s == sf;
            da.Z = opt ? opt->Z : (record ? h->bwd.Z : nullptr);
            da.nc = nc;
            da.mdc = L.mdc;
            RefineArgs& ra = P.ra;
            ra.U = L.Ud; ra.J0 = L.J0; ra.J1w = sb.J1w; ra.Uout = L.U;
            ra.lin = sb.lin;
            ra.stereo = (p.flags & DIS_FLAG_STEREO) ? 1 : 0;
            ra.nc = nc;
            ra.tape = opt ? opt->tape : (record ? h->bwd.tape : nullptr);
            ra.W = W; ra.H = Hh;
            ra.tiles_x = (W + tw - 1) / tw;
            ra.delta = p.w_intensity; ra.gamma = p.w_gradient; ra.alpha = p.w_smooth;
            ra.omega = p.sor_omega; ra.eps = 1e-3;
            for (int q = 0; q < 3; ++q) P.dU[q] = sb.dU[q];
            P.dens_bx = (W + 63) / 64;
            // single-workgroup scales: up to 256 pixel pairs, or up to the
            // block's capacity with the wider setting
            const int small_max = h->small_levels == 2 ? DIS_SMALL_PAIRS : DIS_SMALL_PAIRS / 4;
            // (not in the adjoint's recomputation nor at a scale a forward
            // records for it: the reverse tiles read the tape and the
            // linearisation cache, which only the tiled refinement writes)
            const bool small = p.refine && h->small_levels && !opt && !fbm && nc == 1 && !record &&
                               ((W + 1) / 2) * Hh <= small_max;
            if (small) LH.small.push_back((int)LH.lp.size());
            LH.is_small.push_back(small ? 1 : 0);
            LH.lp.push_back(P);
            const double px = (double)W * Hh;
            const double pxn = s < r.ss ? (double)(r.w >> (s + 1)) * (r.h >> (s + 1)) : 0.0;
            LH.by[0] += search_bytes(px, pxn, N);
            LH.fl[0] += search_flops(N, (double)ps * ps, p.gn_iters);
            const double dby = densify_bytes(px, N, p.refine);
            const double dfl = densify_flops(px, std::pow((double)ps / g.st, 2.0), p.refine);
            if (small) {
                const int nout = p.var_outer < 0 ? s + 1 : p.var_outer;
                LH.sby += dby + 16.0 * px;
                LH.sfl += dfl + nout * refine_flops(px, 2 * p.var_inner);
            } else {
                LH.by[1] += dby;
                LH.fl[1] += dfl;
            }
        }
        levels.push_back(std::move(LH));
    }

    // device tables for every level, one allocation
    size_t bytes = 0;
    int nsync = 0;
    std::vector<size_t> off_lp, off_rph, off_start, off_small, off_fb, off_tseg, off_runs;
    std::vector<int> nruns_of;
    std::vector<int> off_sync;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    // tasks (blocks) of segment (phase ph, pair j) of a level
    // the row-owned search runs one wave per block in its own launch, and
    // 256 threads per task inside the persistent level kernel
    const bool rows = nc == 1 && dis_search_rows_path(&p);
    const int sblock = (rows && mode == 1) ? 64 : 256;
    auto seg_count = [&](const LevelHost& LH, int ph, int j) {
        const LevelPair& P = LH.lp[j];
        if (ph == 0) return (P.sa.nx * P.sa.ny * LH.lpp + sblock - 1) / sblock;
        if (LH.is_small[j]) return 0;   // densified and refined by the single-workgroup launch
        if (ph == 1) return P.dens_bx * ((P.da.H + 3) / 4);
        return P.ra.tiles_x * ((P.ra.H + th - 1) / th);
    };
    for (LevelHost& LH : levels) {
        const int np = (int)LH.lp.size(), nseg = LH.nph * np;
        size_t ntask = 0;
        for (int ph = 0; ph < LH.nph; ++ph)
            for (int j = 0; j < np; ++j) ntask += (size_t)seg_count(LH, ph, j);
        off_tseg.push_back(bytes);
        bytes = al(bytes + sizeof(int) * std::max<size_t>(1, ntask));
        off_runs.push_back(bytes);
        bytes = al(bytes + sizeof(int) * (ntask + 1));
        off_lp.push_back(bytes);
        bytes = al(bytes + sizeof(LevelPair) * np);
        off_rph.push_back(bytes);
        bytes = al(bytes + sizeof(RefPhase) * std::max<size_t>(1, LH.rph.size()));
        off_start.push_back(bytes);
        bytes = al(bytes + sizeof(int) * (nseg + 1));
        off_small.push_back(bytes);
        bytes = al(bytes + sizeof(int) * std::max<size_t>(1, LH.small.size()));
        off_fb.push_back(bytes);
        if (fbm) {
            const LevelPair& P0 = LH.lp[0];
            const size_t ncell = (size_t)((P0.da.W - 1) / ps + 2) * ((P0.da.H - 1) / ps + 2);
            const size_t nlist = (size_t)P0.da.nx * P0.da.ny;
            bytes = al(bytes + 2 * sizeof(int) * (3 * ncell + 1 + nlist));
        }
        off_sync.push_back(nsync);
        tabs.err_index.push_back(nsync + 1);
        nsync += 2 + nseg;
    }
    const int plan_err_index = nsync++;
    const size_t sync_off = bytes;
    bytes += sizeof(int) * nsync;
    if (no_tables) {
        // launches below only take table addresses; with one pair in
        // phase-major order none is dereferenced (LevelLaunch::one)
        tabs.mem = nullptr;
        tabs.bytes = 0;
        tabs.sync = nullptr;
        tabs.nsync = 0;
        tabs.err_index.clear();
    } else {
        HIPCHK(h, hipMalloc(&tabs.mem, bytes));
        tabs.bytes = bytes;
        tabs.sync = (int*)((char*)tabs.mem + sync_off);
        tabs.nsync = nsync;
        tabs.plan_err = tabs.sync + plan_err_index;
    }
    std::vector<char> host(bytes, 0);
    for (size_t li = 0; li < levels.size(); ++li) {
        LevelHost& LH = levels[li];
        const int np = (int)LH.lp.size(), nseg = LH.nph * np;
        std::memcpy(host.data() + off_lp[li], LH.lp.data(), sizeof(LevelPair) * np);
        if (!LH.rph.empty()) std::memcpy(host.data() + off_rph[li], LH.rph.data(), sizeof(RefPhase) * LH.rph.size());
        if (!LH.small.empty())
            std::memcpy(host.data() + off_small[li], LH.small.data(), sizeof(int) * LH.small.size());
        // queue segments, phase-major: search blocks, densification blocks,
        // then the refinement phases, each over all pairs
        std::vector<int> start(nseg + 1, 0);
        std::vector<double> ph_by(LH.nph, 0.0), ph_fl(LH.nph, 0.0);
        ph_by[0] = LH.by[0]; ph_fl[0] = LH.fl[0];
        ph_by[1] = LH.by[1]; ph_fl[1] = LH.fl[1];
        int t = 0;
        for (int ph = 0; ph < LH.nph; ++ph) {
            for (int j = 0; j < np; ++j) {
                const LevelPair& P = LH.lp[j];
                start[ph * np + j] = t;
                const int cnt = seg_count(LH, ph, j);
                int* tseg = (int*)(host.data() + off_tseg[li]) + t;
                for (int q = 0; q < cnt; ++q) tseg[q] = ph * np + j;
                if (ph >= 2 && cnt > 0) {
                    const RefPhase& rp = LH.rph[ph - 2];
                    const double px = (double)P.ra.W * P.ra.H;
                    ph_by[ph] += refine_bytes(px, rp.f >= 0, rp.in >= 0, rp.last);
                    ph_fl[ph] += refine_flops(px, rp.nhalf);
                }
                t += cnt;
            }
        }
        start[nseg] = t;
        std::memcpy(host.data() + off_start[li], start.data(), sizeof(int) * (nseg + 1));
        // runs of the persistent queue: up to rl consecutive tasks of one
        // segment, rl growing with the level's work so that each of the
        // 2 n_cu blocks still takes several runs
        {
            const int rl = std::max(1, std::min(8, t / (8 * h->n_cu)));
            int* rs = (int*)(host.data() + off_runs[li]);
            int nr = 0;
            for (int sg = 0; sg < nseg; ++sg)
                for (int q = start[sg]; q < start[sg + 1]; q += rl) rs[nr++] = q;
            rs[nr] = t;
            nruns_of.push_back(nr);
        }
        LevelLaunch LL;
        std::memset(&LL, 0, sizeof LL);
        if (!no_tables) {
            LL.pairs = (const LevelPair*)((char*)tabs.mem + off_lp[li]);
            LL.rph = (const RefPhase*)((char*)tabs.mem + off_rph[li]);
            LL.start = (const int*)((char*)tabs.mem + off_start[li]);
            LL.task_seg = (const int*)((char*)tabs.mem + off_tseg[li]);
            LL.run_start = (const int*)((char*)tabs.mem + off_runs[li]);
            LL.sync = tabs.sync + off_sync[li];
            LL.plan_err = tabs.plan_err;
        }
        LL.fail_waits = h->fail_waits;
        LL.npairs = np;
        LL.nph = LH.nph;
        LL.ntasks = t;
        LL.nruns = nruns_of[li];
        // the adjoint's reverse tiles read the cache that the recomputation,
        // or a forward recording the finest scale, fills
        LL.lin_cache = (opt || !h->no_lin_cache || (keep_tape && LH.s == sf)) ? 1 : 0;
        if (np == 1) {
            LL.one = 1;
            LL.sa1 = LH.lp[0].sa;
            LL.da1 = LH.lp[0].da;
            LL.dens_bx1 = LH.lp[0].dens_bx;
        }
        if (mode == 0) {
            const void* fn = rows ? dis_kernel_level_rows(ps, LH.lpp, tile_id) : dis_kernel_level(ps, LH.lpp);
            if (!fn) return fail(h, DIS_EINVAL, "no level kernel for patch %d, %d lanes", ps, LH.lpp);
            double by = 0.0, fl = 0.0;
            for (int ph = 0; ph < LH.nph; ++ph) { by += ph_by[ph]; fl += ph_fl[ph]; }
            const int grid = std::max(1, std::min(LL.nruns, h->n_cu * 2));
            seq.add(fn, dim3(grid), dim3(256), &LL, sizeof LL, 0, "level", by, fl);
        } else {
            const void* fs = nc > 1 ? dis_kernel_phase_search_colour(ps)
                             : rows ? dis_kernel_phase_search_rows(ps, LH.lpp) : dis_kernel_phase_search(ps, LH.lpp);
            if (!fs) return fail(h, DIS_EINVAL, "no search kernel for patch %d, %d lanes", ps, LH.lpp);
            for (int ph = 0; ph < LH.nph; ++ph) {
                const int n = start[(ph + 1) * np] - start[ph * np];
                if (n == 0) continue;
                if (ph == 0) {
                    if (opt && opt->skip_search) continue;
                    seq.add(fs, dim3(n), dim3(sblock), &LL, sizeof LL, 0, "search", ph_by[0], ph_fl[0]);
                } else if (ph == 1 && fbm) {
                    // merged densification of both directions (App. B ii):
                    // bin each direction's patches by displaced corner, then gather
                    FbLaunch F;
                    std::memset(&F, 0, sizeof F);
                    F.L = LL;
                    const LevelPair& P0 = LH.lp[0];
                    F.Wc = (P0.da.W - 1) / ps + 2;
                    F.Hc = (P0.da.H - 1) / ps + 2;
                    const size_t ncell = (size_t)F.Wc * F.Hc;
                    const int N = P0.da.nx * P0.da.ny;
                    int* base = (int*)((char*)tabs.mem + off_fb[li]);
                    for (int d = 0; d < 2; ++d) {
                        int* b = base + (size_t)d * (3 * ncell + 1 + N);
                        F.bins[d].count = b;
                        F.bins[d].start = b + ncell;
                        F.bins[d].cursor = b + 2 * ncell + 1;
                        F.bins[d].list = b + 3 * ncell + 1;
                    }
                    const unsigned pb = (unsigned)((N + 255) / 256);
                    seq.add(dis_kernel_fb_count(), dim3(pb, 2), dim3(256), &F, sizeof F, 0, "fb_bin", 16.0 * N, 0.0);
                    seq.add(dis_kernel_fb_scan(), dim3(1, 2), dim3(1024), &F, sizeof F, 0, "fb_bin", 24.0 * ncell, 0.0);
                    seq.add(dis_kernel_fb_scatter(), dim3(pb, 2), dim3(256), &F, sizeof F, 0, "fb_bin", 24.0 * N, 0.0);
                    seq.add(dis_kernel_fb_densify(), dim3((P0.da.W + 63) / 64, (P0.da.H + 3) / 4, 2), dim3(256), &F,
                            sizeof F, 0, "densify", 2.0 * ph_by[1], 2.0 * ph_fl[1]);
                } else if (ph == 1) {
                    seq.add(nc > 1 ? dis_kernel_phase_densify_colour() : dis_kernel_phase_densify(), dim3(n), dim3(256),
                            &LL, sizeof LL, 0, "densify", ph_by[1], ph_fl[1]);
                    if (nc > 1 && p.refine && LH.nph > 2) {
                        // per-channel linearisation of the refinement (one pair per plan)
                        const LevelPair& P0 = LH.lp[0];
                        const double px = (double)P0.ra.W * P0.ra.H;
                        seq.add(dis_kernel_colour_lin(), dim3(P0.dens_bx, (P0.ra.H + 3) / 4), dim3(256), &LL,
                                sizeof LL, 0, "colour_lin", nc * 96.0 * px, nc * 60.0 * px);
                    }
                } else {
                    PhaseLaunch PL;
                    std::memset(&PL, 0, sizeof PL);
                    PL.L = LL;
                    PL.phase = ph;
                    if (LL.one) PL.ra1 = dis_phase_args(LH.lp[0], LH.rph[ph - 2], LL.lin_cache, nc > 1);
                    // (launch-mode bit 6: the lean twin, same core and threads,
                    // where the tiles fill every CU at least twice)
                    const int twin = dis_refine_tile_lean(tile_id);
                    const int tl = (h->lean_big && twin >= 0 && n >= 2 * h->n_cu) ? twin : tile_id;
                    seq.add(nc > 1 ? dis_kernel_phase_refine_colour(tl) : dis_kernel_phase_refine(tl), dim3(n),
                            dim3(nt), &PL, sizeof PL, 0, "refine",
                            ph_by[ph], ph_fl[ph]);
                }
            }
        }
        if (!LH.small.empty()) {
            SmallLaunch SL;
            std::memset(&SL, 0, sizeof SL);
            SL.pairs = LL.pairs;
            SL.list = no_tables ? nullptr : (const int*)((char*)tabs.mem + off_small[li]);
            SL.n = (int)LH.small.size();
            SL.nouter = p.var_outer < 0 ? LH.s + 1 : p.var_outer;
            SL.nhalf = 2 * p.var_inner;
            if (np == 1) {
                SL.da1 = LH.lp[0].da;
                SL.ra1 = LH.lp[0].ra;
            }
            int maxp = 0;
            for (int q : LH.small) maxp = std::max(maxp, (LH.lp[q].ra.W + 1) / 2 * LH.lp[q].ra.H);
            const int snt = maxp <= 512 ? 512 : 1024;   // one pixel pair per thread
            seq.add(dis_kernel_small_level(snt, np == 1), dim3(SL.n), dim3(snt), &SL, sizeof SL, 0, "small_level", LH.sby,
                    LH.sfl);
        }
    }
    if (!no_tables) HIPCHK(h, hipMemcpy(tabs.mem, host.data(), bytes, hipMemcpyHostToDevice));
    return DIS_OK;
}

// Launch sequence of one pair (Alg. 1) into slot `sb`.  Kind 1 launches read
// the caller's frames, kind 2 write the caller's flow.
int dis_build_pair(dis_handle* h, SlotBuf& sb, int w, int hgt, int pitch, const void* I0, const void* I1,
                   void* flow, Seq& seq, PairInfo* info, PlanTables& tabs) {
    const dis_params& p = h->p;
    const int ps = p.patch_size;
    const int ss = dis_coarsest(&p, w, hgt), sf = p.finest_scale;
    if (sf > ss || (w >> sf) < ps || (hgt >> sf) < ps)
        return fail(h, DIS_ESIZE, "%dx%d: scale %d is smaller than the %d px patch", w, hgt, sf, ps);
    if (info) { info->ss = ss; info->sf = sf; }
    const size_t first = seq.items.size();
    int r = dis_add_pyramid(h, sb, w, hgt, pitch, ss, I0, I1, seq);
    if (r != DIS_OK) return r;
    std::vector<PairRef> pr{PairRef{&sb, w, hgt, ss}};
    if (p.flags & DIS_FLAG_FB_CONSISTENCY) pr.push_back(PairRef{&h->slots[1], w, hgt, ss});
    r = dis_build_levels(h, pr, seq, tabs, nullptr);
    if (r != DIS_OK) return r;
    dis_add_upsample(h, sb, w, hgt, flow, tabs.plan_err, seq);
    // the first pyramid launch clears the level launches' queue state
    PyrArgs* pa = (PyrArgs*)seq.items[first].arg.data();
    pa->zero = tabs.sync;
    pa->nzero = tabs.nsync;
    return DIS_OK;
}

// Point the caller-facing launches of a sequence at new frames / flow.
static void rebind(Seq& seq, const void* I0, const void* I1, void* flow) {
    for (Launch& L : seq.items) {
        if (L.kind == 1) {
            PyrArgs* pa = (PyrArgs*)L.arg.data();
            pa->src[0] = I0;
            pa->src[1] = I1;
        } else if (L.kind == 2) {
            ((UpsArgs*)L.arg.data())->out = flow;
        }
    }
}

static int prof_event(dis_handle* h, hipEvent_t* e) {
    if (!h->prof_free.empty()) {
        *e = h->prof_free.back();
        h->prof_free.pop_back();
        return DIS_OK;
    }
    HIPCHK(h, hipEventCreate(e));
    return DIS_OK;
}

// Launch a sequence kernel by kernel.  With profiling on, each run of
// consecutive launches of one kernel family sits between one pair of events
// (so the per-launch average carries one event gap per run, not per launch).
int dis_launch_eager(dis_handle* h, Seq& seq) {
    const size_t n = seq.items.size();
    for (size_t i = 0; i < n;) {
        size_t j = i + 1;
        if (h->profiling)
            while (j < n && std::strcmp(seq.items[j].name, seq.items[i].name) == 0) ++j;
        ProfPending pp{};
        if (h->profiling) {
            int r = prof_event(h, &pp.a);
            if (r == DIS_OK) r = prof_event(h, &pp.b);
            if (r != DIS_OK) return r;
            pp.name = seq.items[i].name;
            pp.launches = (int)(j - i);
            HIPCHK(h, hipEventRecord(pp.a, h->stream));
        }
        for (size_t k = i; k < j; ++k) {
            Launch& L = seq.items[k];
            void* args[1] = {L.arg.data()};
            HIPCHK(h, hipLaunchKernel(L.fn, L.grid, L.block, args, L.shmem, h->stream));
            pp.bytes += L.bytes;
            pp.flops += L.flops;
        }
        if (h->profiling) {
            HIPCHK(h, hipEventRecord(pp.b, h->stream));
            h->prof_pending.push_back(pp);
        }
        i = j;
    }
    return DIS_OK;
}

extern "C" int dis_profile_enable(dis_handle* h, int on) {
    if (!h) return fail(nullptr, DIS_EINVAL, "handle is NULL");
    h->profiling = on != 0;
    return DIS_OK;
}

extern "C" int dis_profile_read(dis_handle* h, dis_kernel_stat* out, int max, int* n) {
    if (!h) return fail(nullptr, DIS_EINVAL, "handle is NULL");
    if (!n || (max > 0 && !out)) return fail(h, DIS_EINVAL, "NULL output");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (ProfPending& pp : h->prof_pending) {
        float ms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&ms, pp.a, pp.b));
        ProfStat& st = h->prof[pp.name];
        st.launches += pp.launches;
        st.ms += ms;
        st.bytes += pp.bytes;
        st.flops += pp.flops;
        h->prof_free.push_back(pp.a);
        h->prof_free.push_back(pp.b);
    }
    h->prof_pending.clear();
    int i = 0;
    for (auto& kv : h->prof) {
        if (i < max) {
            std::memset(&out[i], 0, sizeof out[i]);
            std::snprintf(out[i].name, sizeof out[i].name, "%s", kv.first.c_str());
            out[i].launches = kv.second.launches;
            out[i].total_ms = kv.second.ms;
            out[i].bytes = kv.second.bytes;
            out[i].flops = kv.second.flops;
        }
        ++i;
    }
    *n = i;
    h->prof.clear();
    return DIS_OK;
}

// A graph of one kernel node per launch, chained in order.
int dis_build_graph_seq(dis_handle* h, Seq& seq, hipGraph_t* graph, hipGraphExec_t* exec,
                        std::vector<hipGraphNode_t>* nodes) {
    HIPCHK(h, hipGraphCreate(graph, 0));
    hipGraphNode_t prev = nullptr;
    nodes->resize(seq.items.size());
    for (size_t i = 0; i < seq.items.size(); ++i) {
        Launch& L = seq.items[i];
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof kp);
        void* args[1] = {L.arg.data()};
        kp.func = (void*)L.fn;
        kp.gridDim = L.grid;
        kp.blockDim = L.block;
        kp.sharedMemBytes = (unsigned)L.shmem;
        kp.kernelParams = args;
        kp.extra = nullptr;
        HIPCHK(h, hipGraphAddKernelNode(&(*nodes)[i], *graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
        prev = (*nodes)[i];
    }
    HIPCHK(h, hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0));
    return DIS_OK;
}

// Push the argument blocks of the caller-facing launches (kind != 0) into
// an instantiated graph.
int dis_update_graph_seq(dis_handle* h, Seq& seq, hipGraphExec_t exec, const std::vector<hipGraphNode_t>& nodes) {
    for (size_t i = 0; i < seq.items.size(); ++i) {
        Launch& L = seq.items[i];
        if (L.kind == 0) continue;
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof kp);
        void* args[1] = {L.arg.data()};
        kp.func = (void*)L.fn;
        kp.gridDim = L.grid;
        kp.blockDim = L.block;
        kp.sharedMemBytes = (unsigned)L.shmem;
        kp.kernelParams = args;
        HIPCHK(h, hipGraphExecKernelNodeSetParams(exec, nodes[i], &kp));
    }
    return DIS_OK;
}

static int build_graph(dis_handle* h, Plan* pl) { return dis_build_graph_seq(h, pl->seq, &pl->graph, &pl->exec, &pl->nodes); }

static int update_graph_io(dis_handle* h, Plan* pl) { return dis_update_graph_seq(h, pl->seq, pl->exec, pl->nodes); }

extern "C" int dis_compute_flow(dis_handle* h, const void* I0, const void* I1, int w, int hgt, int pitch,
                                void* flow) {
    if (!h) return fail(nullptr, DIS_EINVAL, "handle is NULL");
    if (!I0 || !I1 || !flow) return fail(h, DIS_EINVAL, "NULL frame or flow pointer");
    if (w < 1 || hgt < 1) return fail(h, DIS_EINVAL, "size %dx%d invalid", w, hgt);
    if (pitch < w) return fail(h, DIS_EINVAL, "pitch %d < width %d", pitch, w);
    if (w > h->max_w || hgt > h->max_h)
        return fail(h, DIS_ESIZE, "%dx%d exceeds the handle's %dx%d", w, hgt, h->max_w, h->max_h);
    const auto key = std::make_tuple(w, hgt, pitch);
    Plan* pl;
    auto it = h->plans.find(key);
    if (it == h->plans.end()) {
        pl = new Plan();
        int r = dis_build_pair(h, h->slots[0], w, hgt, pitch, I0, I1, flow, pl->seq, &pl->info, pl->tabs);
        if (r != DIS_OK) {
            if (pl->tabs.mem) hipFree(pl->tabs.mem);
            delete pl;
            return r;
        }
        h->plans[key] = pl;
    } else {
        pl = it->second;
        rebind(pl->seq, I0, I1, flow);
    }
    int r;
    if ((h->p.flags & DIS_FLAG_NO_GRAPH) || h->profiling) {
        r = dis_launch_eager(h, pl->seq);
    } else {
        if (!pl->exec) {
            r = build_graph(h, pl);
            if (r != DIS_OK) return r;
        } else if (pl->bound[0] != I0 || pl->bound[1] != I1 || pl->bound[2] != flow) {
            r = update_graph_io(h, pl);
            if (r != DIS_OK) return r;
        }
        pl->bound[0] = I0;
        pl->bound[1] = I1;
        pl->bound[2] = flow;
        HIPCHK(h, hipGraphLaunch(pl->exec, h->stream));
        r = DIS_OK;
    }
    if (r == DIS_OK) {
        h->last_w = w;
        h->last_h = hgt;
        h->last_ss = pl->info.ss;
        h->last_sf = pl->info.sf;
        h->have_last = true;
        h->last_I0 = I0;
        h->last_I1 = I1;
        h->last_pitch = pitch;
        h->last_tabs = &pl->tabs;
        h->last_call = 1;
        h->last_flow = flow;
    }
    return r;
}

// --------------------------------------------------------------- debugging

extern "C" int dis_debug_level(dis_handle* h, int s, int what, void* dst, size_t bytes) {
    if (!h) return fail(nullptr, DIS_EINVAL, "handle is NULL");
    if (!dst) return fail(h, DIS_EINVAL, "dst is NULL");
    if (!h->have_last) return fail(h, DIS_ESTATE, "no forward call yet");
    if (what == DIS_DBG_WAIT_ERRORS) {
        // queue-wait timeouts of the last plan's persistent launches
        if (bytes < sizeof(int32_t)) return fail(h, DIS_ESIZE, "need 4 bytes");
        int32_t count = 0;
        const PlanTables* t = h->last_tabs;
        if (t && t->nsync > 0) {
            std::vector<int> sync(t->nsync);
            HIPCHK(h, hipStreamSynchronize(h->stream));
            HIPCHK(h, hipMemcpy(sync.data(), t->sync, sizeof(int) * t->nsync, hipMemcpyDeviceToHost));
            for (int w : t->err_index) count += sync[w] != 0;
        }
        std::memcpy(dst, &count, sizeof count);
        return DIS_OK;
    }
    if (s < h->last_sf || s > h->last_ss) return fail(h, DIS_ESTATE, "scale %d not computed (%d..%d)", s, h->last_sf, h->last_ss);
    LevelBuf& L = h->slots[0].lv[s];
    LevelGrid g;
    const int N = dis_level_grid(h, h->last_w >> s, h->last_h >> s, &g);
    const size_t px = (size_t)g.W * g.H;
    const void* src = nullptr;
    size_t n = 0;
    int32_t info[6];
    switch (what) {
        case DIS_DBG_J0: src = L.J0; n = px * 8; break;
        case DIS_DBG_J1: src = L.J1; n = px * 8; break;
        case DIS_DBG_UINIT: src = L.uinit; n = (size_t)N * 16; break;
        case DIS_DBG_UPATCH: src = nullptr; n = (size_t)N * 16; break;
        case DIS_DBG_UDENSE: src = L.Ud; n = 2 * px * 8; break;
        case DIS_DBG_UREFINED: src = L.U; n = 2 * px * 8; break;
        case DIS_DBG_GRAD_J0: src = h->bwd.gJ0[s]; n = px * 8; break;
        case DIS_DBG_GRAD_J1: src = h->bwd.gJ1[s]; n = px * 8; break;
        case DIS_DBG_GRAD_U: src = h->bwd.gU[s]; n = 2 * px * 8; break;
        case DIS_DBG_GRAD_PATCH: src = h->bwd.gP[s]; n = (size_t)N * 32; break;
        case DIS_DBG_UREFINED_BWD:
            if (!(h->p.flags & DIS_FLAG_FB_CONSISTENCY)) return fail(h, DIS_ESTATE, "not a forward-backward handle");
            src = h->slots[1].lv[s].U; n = 2 * px * 8; break;
        case DIS_DBG_INFO:
            info[0] = g.W; info[1] = g.H; info[2] = N; info[3] = g.nx; info[4] = g.ny; info[5] = g.st;
            if (bytes < sizeof info) return fail(h, DIS_ESIZE, "need %zu bytes", sizeof info);
            std::memcpy(dst, info, sizeof info);
            return DIS_OK;
        default: return fail(h, DIS_EINVAL, "unknown debug item %d", what);
    }
    if (bytes < n) return fail(h, DIS_ESIZE, "need %zu bytes, have %zu", n, bytes);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (what == DIS_DBG_UPATCH) {
        std::vector<double> tmp((size_t)N * 4);
        HIPCHK(h, hipMemcpy(tmp.data(), L.patch, tmp.size() * 8, hipMemcpyDeviceToHost));
        double* o = (double*)dst;
        for (int i = 0; i < N; ++i) { o[2 * i] = tmp[4 * i]; o[2 * i + 1] = tmp[4 * i + 1]; }
        return DIS_OK;
    }
    if (!src) return fail(h, DIS_ESTATE, "item %d not kept at scale %d", what, s);
    HIPCHK(h, hipMemcpy(dst, src, n, hipMemcpyDeviceToHost));
    return DIS_OK;
}
