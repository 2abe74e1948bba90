// Host side of the adjoint: buffers, the per-shape launch plan and
// dis_flow_backward.
//
// The plan walks the scales from fine to coarse.  At each scale it first
// re-runs that scale's densification and refinement from the kept patch
// records (writing the SOR tape and the densification weight sums), then
// runs the reverse of the refinement's fixed-point steps, of the
// densification with the warped frame, and of the inverse search with its
// initialisation from the coarser flow.  Gradients of the level images of
// every scale are summed into the frames by the pyramid adjoint at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dis.h"
#include "dis_backward.h"
#include "dis_host.h"
#include "dis_internal.h"

#define HIPCHK(h, call)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return dis_fail((h), DIS_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define DALLOC(h, ptr, bytes)                                      \
    do {                                                           \
        int r_ = dis_dalloc((h), (void**)&(ptr), (bytes));         \
        if (r_ != DIS_OK) return r_;                               \
    } while (0)

struct BwdPlan {
    Seq seq;
    std::vector<PlanTables> tabs;       // tables of the per-scale recomputation
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> nodes;
    const void* bound[3] = {nullptr, nullptr, nullptr};
};

void dis_bwd_plan_free(BwdPlan* bp) {
    if (!bp) return;
    if (bp->exec) hipGraphExecDestroy(bp->exec);
    if (bp->graph) hipGraphDestroy(bp->graph);
    for (PlanTables& t : bp->tabs)
        if (t.mem) hipFree(t.mem);
    delete bp;
}

static int outer_steps(const dis_params& p, int s) { return p.var_outer < 0 ? s + 1 : p.var_outer; }

// Gradient planes of every processed scale and the scratch of one scale
// (sized for the largest), for slot 0.
int dis_alloc_backward(dis_handle* h) {
    const dis_params& p = h->p;
    BwdBuf& B = h->bwd;
    std::memset(&B, 0, sizeof B);
    const int sf = p.finest_scale;
    size_t tape = 0, pxmax = 0;
    for (int s = sf; s <= h->top; ++s) {
        const LevelBuf& L = h->slots[0].lv[s];
        if (!L.U) continue;
        const size_t px = (size_t)(h->max_w >> s) * (h->max_h >> s);
        DALLOC(h, B.gJ0[s], px * sizeof(double));
        DALLOC(h, B.gJ1[s], px * sizeof(double));
        DALLOC(h, B.gU[s], 2 * px * sizeof(double));
        DALLOC(h, B.gP[s], (size_t)L.maxN * 4 * sizeof(double));
        pxmax = std::max(pxmax, px);
        if (p.refine) tape = std::max(tape, ((size_t)outer_steps(p, s) * 2 * p.var_inner + 1) * 2 * px);
    }
    B.scratch_px = pxmax;
    DALLOC(h, B.Z, pxmax * sizeof(double));
    if (p.refine) {
        DALLOC(h, B.gUd, 2 * pxmax * sizeof(double));
        DALLOC(h, B.gJ1w, pxmax * sizeof(double));
        DALLOC(h, B.gd, 2 * pxmax * sizeof(double));
        DALLOC(h, B.gn, 2 * pxmax * sizeof(double));
        DALLOC(h, B.acc, 9 * pxmax * sizeof(double));
        DALLOC(h, B.coef, 6 * pxmax * sizeof(double));
        DALLOC(h, B.edge, 4 * pxmax * sizeof(double));
        DALLOC(h, B.gFacc, 2 * pxmax * sizeof(double));
        DALLOC(h, B.tape, tape * sizeof(double));
        B.tape_len = tape;
    }
    return DIS_OK;
}

static void add_zero(Seq& q, double* p, size_t n) {
    BZeroArgs z{p, n};
    q.add(dis_kernel_bzero(), dim3((unsigned)((n + 255) / 256)), dim3(256), &z, sizeof z, 0, "bwd_zero", 8.0 * n, 0.0);
}

static dim3 grid2d(int W, int H) { return dim3((W + 63) / 64, (H + 3) / 4); }

static int build_backward(dis_handle* h, int w, int hgt, BwdPlan* bp) {
    const dis_params& p = h->p;
    BwdBuf& B = h->bwd;
    SlotBuf& sb = h->slots[0];
    const int ps = p.patch_size, sf = p.finest_scale;
    const int ss = dis_coarsest(&p, w, hgt);
    const int cmap = (p.flags & DIS_FLAG_PIXEL_CENTRE) ? 1 : 0;
    const bool f64io = (p.flags & DIS_FLAG_IO_F64) != 0;
    const size_t shmem = (size_t)16 * (p.gn_iters + 1) * 2 * sizeof(double);
    if (shmem > 65536) return dis_fail(h, DIS_EINVAL, "backward supports at most 255 Gauss-Newton iterations");
    Seq& q = bp->seq;

    for (int s = sf; s <= ss; ++s) {
        LevelGrid g;
        const int N = dis_level_grid(h, w >> s, hgt >> s, &g);
        const size_t n = (size_t)g.W * g.H;
        add_zero(q, B.gJ0[s], n);
        add_zero(q, B.gJ1[s], n);
        add_zero(q, B.gU[s], 2 * n);
        add_zero(q, B.gP[s], (size_t)N * 4);
    }
    {
        UpsBwdArgs ua;
        std::memset(&ua, 0, sizeof ua);
        ua.gF = nullptr;   // bound per call
        ua.g_f64 = f64io ? 1 : 0;
        ua.W = w;
        ua.H = hgt;
        ua.f = (double)(1 << sf);
        ua.centre_map = cmap;
        ua.gU = B.gU[sf];
        ua.Ws = w >> sf;
        ua.Hs = hgt >> sf;
        q.add(dis_kernel_bwd_upsample(), grid2d(w, hgt), dim3(256), &ua, sizeof ua, 3, "bwd_upsample",
              (f64io ? 16.0 : 8.0) * w * hgt + 16.0 * ua.Ws * ua.Hs, 20.0 * w * hgt);
    }

    for (int s = sf; s <= ss; ++s) {
        LevelBuf& L = sb.lv[s];
        LevelGrid g;
        const int N = dis_level_grid(h, w >> s, hgt >> s, &g);
        const int W = g.W, H = g.H;
        const size_t n = (size_t)W * H;
        const double px = (double)n;

        // recompute densification and refinement of this scale
        LevelOpts o;
        o.only_level = s;
        o.tape = p.refine ? B.tape : nullptr;
        o.Z = B.Z;
        o.skip_search = 1;
        o.force_phase = 1;
        bp->tabs.emplace_back();
        std::vector<PairRef> pr{PairRef{&sb, w, hgt, ss}};
        int r = dis_build_levels(h, pr, q, bp->tabs.back(), &o);
        if (r != DIS_OK) return r;

        const double* gUd = B.gU[s];
        const double* gJ1w = nullptr;
        if (p.refine) {
            BCopyArgs cp{B.gUd, B.gU[s], B.gd, 2 * n};
            q.add(dis_kernel_bcopy(), dim3((unsigned)((2 * n + 255) / 256)), dim3(256), &cp, sizeof cp, 0, "bwd_copy",
                  48.0 * n, 0.0);
            add_zero(q, B.gJ1w, n);
            gUd = B.gUd;
            gJ1w = B.gJ1w;
            const int nout = outer_steps(p, s);
            const int nh = 2 * p.var_inner;
            for (int k = nout - 1; k >= 0; --k) {
                RefBwdArgs ra;
                std::memset(&ra, 0, sizeof ra);
                ra.U = L.Ud;
                ra.F = k ? B.tape + (size_t)k * nh * 2 * n : nullptr;
                ra.J0 = L.J0;
                ra.J1w = sb.J1w;
                ra.coef = B.coef;
                ra.acc = B.acc;
                ra.edge = B.edge;
                ra.gU = B.gUd;
                ra.gF = B.gFacc;
                ra.gJ0 = B.gJ0[s];
                ra.gJ1w = B.gJ1w;
                ra.W = W;
                ra.H = H;
                ra.delta = p.w_intensity;
                ra.gamma = p.w_gradient;
                ra.alpha = p.w_smooth;
                ra.omega = p.sor_omega;
                ra.eps = 1e-3;
                q.add(dis_kernel_bwd_coef(), grid2d(W, H), dim3(256), &ra, sizeof ra, 0, "bwd_coef", 40.0 * px,
                      20.0 * px);
                q.add(dis_kernel_bwd_coef2(), grid2d(W, H), dim3(256), &ra, sizeof ra, 0, "bwd_coef", 88.0 * px,
                      120.0 * px);
                add_zero(q, B.acc, 9 * n);
                if (k) add_zero(q, B.gFacc, 2 * n);
                for (int j = nh - 1; j >= 0; --j) {
                    const int m = k * nh + j;
                    SweepBwdArgs sw;
                    std::memset(&sw, 0, sizeof sw);
                    sw.state = m ? B.tape + (size_t)m * 2 * n : nullptr;
                    sw.coef = B.coef;
                    sw.gd = B.gd;
                    sw.gn = B.gn;
                    sw.acc = B.acc;
                    sw.W = W;
                    sw.H = H;
                    sw.colour = j & 1;
                    sw.omega = p.sor_omega;
                    q.add(dis_kernel_bwd_sweep_a(), grid2d(W, H), dim3(256), &sw, sizeof sw, 0, "bwd_sweep",
                          0.5 * 232.0 * px, 0.5 * 60.0 * px);
                    q.add(dis_kernel_bwd_sweep_b(), grid2d(W, H), dim3(256), &sw, sizeof sw, 0, "bwd_sweep",
                          0.5 * 80.0 * px, 0.5 * 16.0 * px);
                }
                q.add(dis_kernel_bwd_lin(), grid2d(W, H), dim3(256), &ra, sizeof ra, 0, "bwd_lin", 200.0 * px,
                      400.0 * px);
                q.add(dis_kernel_bwd_ws(), grid2d(W, H), dim3(256), &ra, sizeof ra, 0, "bwd_ws", 96.0 * px,
                      60.0 * px);
                if (k) {
                    BCopyArgs ax{B.gd, B.gFacc, nullptr, 2 * n};
                    q.add(dis_kernel_baxpy(), dim3((unsigned)((2 * n + 255) / 256)), dim3(256), &ax, sizeof ax, 0,
                          "bwd_copy", 48.0 * n, 2.0 * n);
                }
            }
        }

        DensBwdArgs da;
        std::memset(&da, 0, sizeof da);
        da.J0 = L.J0;
        da.J1 = L.J1;
        da.W = W;
        da.H = H;
        da.patch = L.patch;
        da.ps = ps;
        da.st = g.st;
        da.nrx = g.nrx;
        da.nry = g.nry;
        da.nx = g.nx;
        da.ny = g.ny;
        da.raw_residual = (p.flags & DIS_FLAG_RAW_RESIDUAL) ? 1 : 0;
        da.Ud = L.Ud;
        da.Z = B.Z;
        da.gUd = gUd;
        da.gJ1w = gJ1w;
        da.gJ0 = B.gJ0[s];
        da.gJ1 = B.gJ1[s];
        da.gP = B.gP[s];
        const double cover = std::pow((double)ps / g.st, 2.0);
        q.add(dis_kernel_bwd_densify(), grid2d(W, H), dim3(256), &da, sizeof da, 0, "bwd_densify",
              72.0 * px + 32.0 * N, cover * 60.0 * px);

        SearchBwdArgs sa;
        std::memset(&sa, 0, sizeof sa);
        SearchArgs& a = sa.sa;
        a.J0 = L.J0;
        a.J1 = L.J1;
        a.W = W;
        a.H = H;
        if (s < ss) {
            a.Un = sb.lv[s + 1].U;
            a.Wn = w >> (s + 1);
            a.Hn = hgt >> (s + 1);
            sa.gUn = B.gU[s + 1];
        }
        a.st = g.st;
        a.nrx = g.nrx;
        a.nry = g.nry;
        a.nx = g.nx;
        a.ny = g.ny;
        a.iters = p.gn_iters;
        a.lam = 1e-3;
        a.centre_map = cmap;
        a.patch = L.patch;
        a.uinit = L.uinit;
        sa.gP = B.gP[s];
        sa.gJ0 = B.gJ0[s];
        sa.gJ1 = B.gJ1[s];
        const void* fs = dis_kernel_bwd_search(ps);
        if (!fs) return dis_fail(h, DIS_EINVAL, "no backward search kernel for patch %d", ps);
        const unsigned nb = (unsigned)(((size_t)N * 16 + 255) / 256);
        q.add(fs, dim3(nb), dim3(256), &sa, sizeof sa, 0, "bwd_search", 16.0 * px + 64.0 * N,
              (double)N * ps * ps * (2.0 * p.gn_iters + 1.0) * 40.0);
        q.items.back().shmem = shmem;
    }

    PyrBwdArgs pa;
    std::memset(&pa, 0, sizeof pa);
    for (int s = 0; s < DIS_MAXL; ++s) {
        pa.ws[s] = w >> s;
        pa.hs[s] = hgt >> s;
        if (s >= sf && s <= ss) {
            pa.gJ0[s] = B.gJ0[s];
            pa.gJ1[s] = B.gJ1[s];
        }
    }
    pa.sf = sf;
    pa.ss = ss;
    pa.W = w;
    pa.H = hgt;
    pa.out_f64 = f64io ? 1 : 0;
    double pyb = 0.0;
    for (int s = sf; s <= ss; ++s) pyb += 16.0 * (double)(w >> s) * (hgt >> s);
    q.add(dis_kernel_bwd_pyramid(), grid2d(w, hgt), dim3(256), &pa, sizeof pa, 4, "bwd_pyramid",
          pyb + (f64io ? 16.0 : 8.0) * w * hgt, 4.0 * (ss - sf + 1) * w * hgt);
    return DIS_OK;
}

static void bind_backward(BwdPlan* bp, const void* gF, void* gI0, void* gI1) {
    for (Launch& L : bp->seq.items) {
        if (L.kind == 3) {
            ((UpsBwdArgs*)L.arg.data())->gF = gF;
        } else if (L.kind == 4) {
            PyrBwdArgs* pa = (PyrBwdArgs*)L.arg.data();
            pa->gI0 = gI0;
            pa->gI1 = gI1;
        }
    }
}

extern "C" int dis_flow_backward(dis_handle* h, const void* grad_flow, void* grad_I0, void* grad_I1) {
    if (!h) return dis_fail(nullptr, DIS_EINVAL, "handle is NULL");
    if (!grad_flow || !grad_I0 || !grad_I1) return dis_fail(h, DIS_EINVAL, "NULL gradient pointer");
    if (!(h->p.flags & DIS_FLAG_KEEP_FOR_BACKWARD))
        return dis_fail(h, DIS_ESTATE, "the handle was created without DIS_FLAG_KEEP_FOR_BACKWARD");
    if (!h->have_last || h->last_call != 1)
        return dis_fail(h, DIS_ESTATE, "no dis_compute_flow call to differentiate (a batched call replaces it)");
    const int w = h->last_w, hgt = h->last_h;
    const auto key = std::make_tuple(w, hgt);
    BwdPlan* bp;
    auto it = h->bwplans.find(key);
    if (it == h->bwplans.end()) {
        bp = new BwdPlan();
        int r = build_backward(h, w, hgt, bp);
        if (r != DIS_OK) {
            dis_bwd_plan_free(bp);
            return r;
        }
        h->bwplans[key] = bp;
    } else {
        bp = it->second;
    }
    bind_backward(bp, grad_flow, grad_I0, grad_I1);
    if ((h->p.flags & DIS_FLAG_NO_GRAPH) || h->profiling) return dis_launch_eager(h, bp->seq);
    if (!bp->exec) {
        int r = dis_build_graph_seq(h, bp->seq, &bp->graph, &bp->exec, &bp->nodes);
        if (r != DIS_OK) return r;
    } else if (bp->bound[0] != grad_flow || bp->bound[1] != grad_I0 || bp->bound[2] != grad_I1) {
        int r = dis_update_graph_seq(h, bp->seq, bp->exec, bp->nodes);
        if (r != DIS_OK) return r;
    }
    bp->bound[0] = grad_flow;
    bp->bound[1] = grad_I0;
    bp->bound[2] = grad_I1;
    HIPCHK(h, hipGraphLaunch(bp->exec, h->stream));
    return DIS_OK;
}
