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
    DALLOC(h, B.gq, 2 * pxmax * sizeof(double));
    if (p.refine) {
        DALLOC(h, B.gUd, 2 * pxmax * sizeof(double));
        DALLOC(h, B.gJ1w, pxmax * sizeof(double));
        DALLOC(h, B.gd, 2 * pxmax * sizeof(double));
        DALLOC(h, B.gn, 2 * pxmax * sizeof(double));
        DALLOC(h, B.acc, 9 * pxmax * sizeof(double));
        DALLOC(h, B.coef, 6 * pxmax * sizeof(double));
        int nout_max = 1;
        for (int s = sf; s <= h->top; ++s) nout_max = std::max(nout_max, outer_steps(p, s));
        DALLOC(h, B.gFacc, (size_t)nout_max * 2 * pxmax * sizeof(double));
        DALLOC(h, B.tape, tape * sizeof(double));
        B.tape_len = tape;
    }
    return DIS_OK;
}


static dim3 grid2d(int W, int H) { return dim3((W + 63) / 64, (H + 3) / 4); }

// Clear many buffers with as few launches as possible (eight per launch).
static void add_zero_list(Seq& q, const std::vector<std::pair<double*, size_t>>& bufs) {
    for (size_t i0 = 0; i0 < bufs.size(); i0 += 8) {
        BZeroList z;
        std::memset(&z, 0, sizeof z);
        int blocks = 0;
        double bytes = 0.0;
        for (size_t i = i0; i < bufs.size() && i < i0 + 8; ++i) {
            if (bufs[i].second == 0) continue;
            z.p[z.cnt] = bufs[i].first;
            z.n[z.cnt] = bufs[i].second;
            z.start[z.cnt] = blocks;
            blocks += (int)((bufs[i].second + 255) / 256);
            bytes += 8.0 * bufs[i].second;
            ++z.cnt;
        }
        z.start[z.cnt] = blocks;
        if (z.cnt) q.add(dis_kernel_bzero_list(), dim3(blocks), dim3(256), &z, sizeof z, 0, "bwd_zero", bytes, 0.0);
    }
}

// Reverse refinement tile of a W x H scale.  Scales with at least one
// 16x16 tile per two compute units take 16x16 cores over 5 half sweeps per
// launch: a region of 28x28 per core of 256 pixels, against 30x30 per 64
// for 8x8 cores over 10 (twice the launches, a third of the halo work).
// Smaller scales take 8x8 cores over 10 half sweeps, which keep more
// blocks in flight.  (8 pairs of 512x256: 5.91 ms forward+backward, against
// 6.39 with 16x16 cores over 10 half sweeps on the two finest scales.)
static int bwd_step_pick(const dis_handle* h, int W, int H) {
    return 2 * ((W + 15) / 16) * ((H + 15) / 16) >= h->n_cu ? 1 : 0;
}

static int build_backward(dis_handle* h, int w, int hgt, BwdPlan* bp) {
    const dis_params& p = h->p;
    BwdBuf& B = h->bwd;
    SlotBuf& sb = h->slots[0];
    const int ps = p.patch_size, sf = p.finest_scale;
    const int ss = dis_coarsest(&p, w, hgt);
    const int cmap = (p.flags & DIS_FLAG_PIXEL_CENTRE) ? 1 : 0;
    const bool f64io = (p.flags & DIS_FLAG_IO_F64) != 0;
    // search reverse: iterates of 16 patches, then one or two LDS windows
    // per patch (J1 adjoint, J1 values), as wide as 64 KB of LDS allows
    // (PS + 3 to PS + 15 cells a side)
    const size_t traj = (size_t)16 * (p.gn_iters + 1) * 2 * sizeof(double);
    const size_t wbytes = (size_t)16 * 8 * dis_bwd_search_windows(ps);
    if (traj > 65536 - wbytes * (ps + 3) * (ps + 3))
        return dis_fail(h, DIS_EINVAL, "backward supports at most %d Gauss-Newton iterations for patch %d",
                        (int)((65536 - wbytes * (ps + 3) * (ps + 3)) / (16 * 2 * 8)) - 1, ps);
    int win = ps + 15;
    while (win > ps + 3 && traj + wbytes * win * win > 65536) --win;
    const size_t shmem = traj + wbytes * win * win;
    Seq& q = bp->seq;

    {
        std::vector<std::pair<double*, size_t>> z;
        for (int s = sf; s <= ss; ++s) {
            LevelGrid g;
            const int N = dis_level_grid(h, w >> s, hgt >> s, &g);
            const size_t n = (size_t)g.W * g.H;
            z.push_back({B.gJ0[s], n});
            z.push_back({B.gJ1[s], n});
            z.push_back({B.gU[s], 2 * n});
            z.push_back({B.gP[s], (size_t)N * 4});
        }
        add_zero_list(q, z);
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

        // recompute densification and refinement of this scale; the finest
        // scale's weight sums, tape, warped frame and linearisation are still
        // those the forward left (it recorded them)
        if (s != sf || !dis_forward_keeps_finest(h)) {
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
        }

        const double* gUd = B.gU[s];
        const double* gJ1w = nullptr;
        if (p.refine) {
            const int nout = outer_steps(p, s);
            const int nh = 2 * p.var_inner;
            const bool tiled = !h->bwd_reference;
            BCopyArgs cp{B.gUd, B.gU[s], B.gd, 2 * n};
            q.add(dis_kernel_bcopy(), dim3((unsigned)((2 * n + 255) / 256)), dim3(256), &cp, sizeof cp, 0, "bwd_copy",
                  48.0 * n, 0.0);
            {
                std::vector<std::pair<double*, size_t>> z{{B.gJ1w, n}};
                if (tiled)
                    for (int k = 1; k < nout; ++k) z.push_back({B.gFacc + (size_t)k * 2 * n, 2 * n});
                add_zero_list(q, z);
            }
            gUd = B.gUd;
            gJ1w = B.gJ1w;
            // adjoint of the state between half sweeps: ping-pong between gd and gn
            double* gdb[2] = {B.gd, B.gn};
            int cur = 0;
            const int shape = bwd_step_pick(h, W, H);
            int TW = 8, TH = 8, KH = 1;
            if (!dis_bwd_step_shape(shape, &TW, &TH, &KH)) return dis_fail(h, DIS_EINVAL, "internal: reverse tile %d", shape);
            const int tiles_x = (W + TW - 1) / TW;
            const int ntiles = tiles_x * ((H + TH - 1) / TH);
            for (int k = nout - 1; k >= 0; --k) {
                RefBwdArgs ra;
                std::memset(&ra, 0, sizeof ra);
                ra.U = L.Ud;
                ra.F = k ? B.tape + (size_t)k * nh * 2 * n : nullptr;
                ra.J0 = L.J0;
                ra.J1w = sb.J1w;
                ra.coef = B.coef;
                ra.acc = B.acc;
                ra.gU = B.gUd;
                ra.gF = tiled ? (k ? B.gFacc + (size_t)k * 2 * n : nullptr) : B.gFacc;
                ra.gJ0 = B.gJ0[s];
                ra.gJ1w = B.gJ1w;
                ra.W = W;
                ra.H = H;
                ra.delta = p.w_intensity;
                ra.gamma = p.w_gradient;
                ra.alpha = p.w_smooth;
                ra.omega = p.sor_omega;
                ra.eps = 1e-3;
                if (tiled) {
                    // reverse of the step's half sweeps, at most KH per launch
                    int j_hi = nh;
                    bool first = true;
                    while (j_hi > 0) {
                        const int j_lo = std::max(0, j_hi - KH);
                        BwdStepArgs st;
                        std::memset(&st, 0, sizeof st);
                        RefineArgs& f = st.ra;
                        f.U = L.Ud;
                        f.J0 = L.J0;
                        f.J1w = sb.J1w;
                        f.lin = sb.lin;
                        f.lin_mode = 2;   // filled by the recomputation's first refinement launch
                        f.dUf = ra.F;
                        f.W = W;
                        f.H = H;
                        f.nhalf = j_hi - j_lo;
                        f.tiles_x = tiles_x;
                        f.delta = p.w_intensity;
                        f.gamma = p.w_gradient;
                        f.alpha = p.w_smooth;
                        f.omega = p.sor_omega;
                        f.eps = 1e-3;
                        st.tape = B.tape;
                        st.m0 = k * nh;
                        st.j_lo = j_lo;
                        st.j_hi = j_hi;
                        st.gd_in = gdb[cur];
                        st.gadd = (first && k < nout - 1) ? B.gFacc + (size_t)(k + 1) * 2 * n : nullptr;
                        st.gd_out = gdb[cur ^ 1];
                        st.coef = B.coef;
                        st.acc = B.acc;
                        st.acc_load = first ? 0 : 1;
                        const int kh = j_hi - j_lo;
                        // in: U, dUf, J0, J1w, state adjoint (+ added), kh tape states;
                        // out: state adjoint, 9 coefficient adjoints, 3 coefficients
                        q.add(dis_kernel_bwd_step(shape), dim3(ntiles), dim3(DIS_BWD_THREADS), &st, sizeof st, 0,
                              "bwd_step", px * (16.0 + 16.0 + 16.0 + 32.0 + 16.0 * kh + 16.0 + 72.0 + 24.0),
                              px * (155.0 + 20.0 * kh));
                        cur ^= 1;
                        first = false;
                        j_hi = j_lo;
                    }
                } else {
                    q.add(dis_kernel_bwd_coef(), grid2d(W, H), dim3(256), &ra, sizeof ra, 0, "bwd_coef", 40.0 * px,
                          20.0 * px);
                    q.add(dis_kernel_bwd_coef2(), grid2d(W, H), dim3(256), &ra, sizeof ra, 0, "bwd_coef", 88.0 * px,
                          120.0 * px);
                    add_zero_list(q, {{B.acc, 9 * n}, {B.gFacc, k ? 2 * n : 0}});
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
                }
                q.add(dis_kernel_bwd_lin_ws(), grid2d(W, H), dim3(256), &ra, sizeof ra, 0, "bwd_lin", 232.0 * px,
                      460.0 * px);
                if (!tiled && k) {
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
        da.gq = B.gq;
        const double cover = std::pow((double)ps / g.st, 2.0);
        q.add(dis_kernel_bwd_densify(), grid2d(W, H), dim3(256), &da, sizeof da, 0, "bwd_densify",
              72.0 * px, cover * 40.0 * px);
        q.add(dis_kernel_bwd_densify_patch(), dim3((unsigned)((N * 16 + 255) / 256)), dim3(256), &da, sizeof da, 0,
              "bwd_densify", 64.0 * px + 32.0 * N, cover * 40.0 * px);

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
        sa.win = win;
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
    if (h->p.flags & DIS_FLAG_STEREO)
        return dis_fail(h, DIS_EINVAL, "the adjoint covers two-dimensional flow, not the stereo form");
    if (h->p.flags & DIS_FLAG_FB_CONSISTENCY)
        return dis_fail(h, DIS_EINVAL, "the adjoint covers the one-directional densification, not the merged one");
    if (h->p.flags & DIS_FLAG_COLOUR) return dis_fail(h, DIS_EINVAL, "the adjoint covers grey frames");
    if (h->p.norm != DIS_NORM_L2)
        return dis_fail(h, DIS_EINVAL, "the adjoint covers the L2 inverse search (norm %d requested)", h->p.norm);
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
