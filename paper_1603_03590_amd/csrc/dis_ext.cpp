// Batched flow, the launch-choice autotuner and the backward entry point.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dis.h"
#include "dis_host.h"
#include "dis_internal.h"

#define XHIPCHK(h, call)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return dis_fail((h), DIS_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

// ------------------------------------------------------------------ batched

// A batch composition's launch plan: multi-pair pyramid passes, the level
// launches over every pair, one multi-pair upscaling.  The caller's frame and
// flow pointers live only in the device tables of the first pyramid pass and
// of the upscaling, so a new set of pointers is one table upload.
struct BatchPlan {
    Seq seq;
    PlanTables tabs;
    void* io = nullptr;                 // device: pyramid tables, upscaling table, start arrays
    size_t pyr0_off = 0, ups_off = 0;
    std::vector<PyrArgs> pyr0;          // host copy of the first pass's table
    std::vector<UpsArgs> ups;           // host copy of the upscaling table
    std::vector<const void*> bound;     // I0, I1, flow of every pair, as uploaded
    std::vector<int> ss;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

void dis_batch_plan_free(BatchPlan* bp) {
    if (!bp) return;
    if (bp->exec) hipGraphExecDestroy(bp->exec);
    if (bp->graph) hipGraphDestroy(bp->graph);
    if (bp->tabs.mem) hipFree(bp->tabs.mem);
    if (bp->io) hipFree(bp->io);
    delete bp;
}

static int build_batch(dis_handle* h, int n, const int* w, const int* hgt, const int* pitch, BatchPlan* bp) {
    const dis_params& p = h->p;
    const int ps = p.patch_size, sf = p.finest_scale;
    const bool f64io = (p.flags & DIS_FLAG_IO_F64) != 0;
    std::vector<PairRef> pairs;
    int top = 0;
    for (int k = 0; k < n; ++k) {
        const int ss = dis_coarsest(&p, w[k], hgt[k]);
        if (sf > ss || (w[k] >> sf) < ps || (hgt[k] >> sf) < ps)
            return dis_fail(h, DIS_ESIZE, "pair %d (%dx%d): scale %d is smaller than the %d px patch", k, w[k], hgt[k],
                            sf, ps);
        pairs.push_back(PairRef{&h->slots[k], w[k], hgt[k], ss});
        bp->ss.push_back(ss);
        top = std::max(top, ss);
    }
    // pyramid passes a = 0, 5, 10, ...: one launch per pass over the pairs that need it
    std::vector<std::vector<PyrArgs>> passes;
    std::vector<std::vector<int>> pstart;
    for (int a = 0; a < top || a == 0; a += 5) {
        Seq tmp;
        std::vector<PyrArgs> tab;
        std::vector<int> st{0};
        for (int k = 0; k < n; ++k) {
            if (a > 0 && pairs[k].ss <= a) continue;
            tmp.items.clear();
            dis_add_pyramid(h, *pairs[k].sb, w[k], hgt[k], pitch[k], pairs[k].ss, nullptr, nullptr, tmp);
            const size_t idx = (size_t)a / 5;
            if (idx >= tmp.items.size()) continue;
            const PyrArgs pa = *(const PyrArgs*)tmp.items[idx].arg.data();
            tab.push_back(pa);
            st.push_back(st.back() + dis_pyramid_tiles(pa));
        }
        if (tab.empty()) break;
        passes.push_back(tab);
        pstart.push_back(st);
        if (top == 0) break;
    }
    bp->pyr0 = passes[0];
    // upscaling table
    std::vector<int> ust{0};
    for (int k = 0; k < n; ++k) {
        Seq tmp;
        dis_add_upsample(h, *pairs[k].sb, w[k], hgt[k], nullptr, nullptr, tmp);
        const UpsArgs ua = *(const UpsArgs*)tmp.items[0].arg.data();
        bp->ups.push_back(ua);
        ust.push_back(ust.back() + ((w[k] + 255) / 256) * dis_upsample_blocks_y(w[k], hgt[k]));
    }
    // device layout of the pyramid and upscaling tables
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t bytes = 0;
    std::vector<size_t> off_tab, off_st;
    // block -> pair maps (one load per block instead of a search of start[])
    auto block_map = [](const std::vector<int>& st) {
        std::vector<int> m(st.back());
        for (size_t j = 0; j + 1 < st.size(); ++j)
            for (int t = st[j]; t < st[j + 1]; ++t) m[t] = (int)j;
        return m;
    };
    std::vector<size_t> off_map;
    std::vector<std::vector<int>> pmaps;
    for (size_t i = 0; i < passes.size(); ++i) {
        off_tab.push_back(bytes);
        bytes = al(bytes + sizeof(PyrArgs) * passes[i].size());
        off_st.push_back(bytes);
        bytes = al(bytes + sizeof(int) * pstart[i].size());
        pmaps.push_back(block_map(pstart[i]));
        off_map.push_back(bytes);
        bytes = al(bytes + sizeof(int) * pmaps.back().size());
    }
    bp->ups_off = bytes;
    bytes = al(bytes + sizeof(UpsArgs) * n);
    const size_t ust_off = bytes;
    bytes = al(bytes + sizeof(int) * (n + 1));
    const std::vector<int> umap = block_map(ust);
    const size_t umap_off = bytes;
    bytes = al(bytes + sizeof(int) * umap.size());
    XHIPCHK(h, hipMalloc(&bp->io, bytes));
    bp->pyr0_off = off_tab[0];

    // launches: pyramid passes, levels, upscaling
    const size_t first = bp->seq.items.size();
    for (size_t i = 0; i < passes.size(); ++i) {
        PyrTab T;
        std::memset(&T, 0, sizeof T);
        T.tab = (const PyrArgs*)((char*)bp->io + off_tab[i]);
        T.start = (const int*)((char*)bp->io + off_st[i]);
        T.blk = (const int*)((char*)bp->io + off_map[i]);
        T.n = (int)passes[i].size();
        double by = 0.0;
        for (const PyrArgs& pa : passes[i]) by += 2.0 * pa.w0 * pa.h0 * (i == 0 ? (f64io ? 8 : 4) : 8);
        bp->seq.add(dis_kernel_pyramid_tab(), dim3(pstart[i].back(), 2), dim3(DIS_PYR_THREADS), &T, sizeof T, 0, "pyramid", by,
                    0.0);
    }
    int r = dis_build_levels(h, pairs, bp->seq, bp->tabs, nullptr);
    if (r != DIS_OK) return r;
    {
        PyrTab* T0 = (PyrTab*)bp->seq.items[first].arg.data();
        T0->zero = bp->tabs.sync;
        T0->nzero = bp->tabs.nsync;
    }
    // a persistent wait that gives up turns every flow of the batch into NaN
    for (UpsArgs& ua : bp->ups) ua.poison = bp->tabs.plan_err;
    UpsTab UT;
    std::memset(&UT, 0, sizeof UT);
    UT.tab = (const UpsArgs*)((char*)bp->io + bp->ups_off);
    UT.start = (const int*)((char*)bp->io + ust_off);
    UT.blk = (const int*)((char*)bp->io + umap_off);
    UT.n = n;
    double uby = 0.0;
    for (int k = 0; k < n; ++k) uby += (f64io ? 16.0 : 8.0) * w[k] * hgt[k];
    bp->seq.add(dis_kernel_upsample_tab(), dim3(ust.back()), dim3(256), &UT, sizeof UT, 0, "upsample", uby,
                20.0 * uby / 8.0);

    std::vector<char> host(bytes, 0);
    for (size_t i = 0; i < passes.size(); ++i) {
        std::memcpy(host.data() + off_tab[i], passes[i].data(), sizeof(PyrArgs) * passes[i].size());
        std::memcpy(host.data() + off_st[i], pstart[i].data(), sizeof(int) * pstart[i].size());
        std::memcpy(host.data() + off_map[i], pmaps[i].data(), sizeof(int) * pmaps[i].size());
    }
    std::memcpy(host.data() + umap_off, umap.data(), sizeof(int) * umap.size());
    std::memcpy(host.data() + bp->ups_off, bp->ups.data(), sizeof(UpsArgs) * n);
    std::memcpy(host.data() + ust_off, ust.data(), sizeof(int) * (n + 1));
    XHIPCHK(h, hipMemcpy(bp->io, host.data(), bytes, hipMemcpyHostToDevice));
    bp->bound.assign(3 * n, nullptr);
    return DIS_OK;
}

static int build_batch_graph(dis_handle* h, BatchPlan* bp) {
    XHIPCHK(h, hipGraphCreate(&bp->graph, 0));
    hipGraphNode_t prev = nullptr;
    for (Launch& L : bp->seq.items) {
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof kp);
        void* args[1] = {L.arg.data()};
        kp.func = (void*)L.fn;
        kp.gridDim = L.grid;
        kp.blockDim = L.block;
        kp.kernelParams = args;
        hipGraphNode_t node;
        XHIPCHK(h, hipGraphAddKernelNode(&node, bp->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
        prev = node;
    }
    XHIPCHK(h, hipGraphInstantiate(&bp->exec, bp->graph, nullptr, nullptr, 0));
    return DIS_OK;
}

extern "C" int dis_compute_flow_batched(dis_handle* h, int n, const void* const* I0, const void* const* I1,
                                        const int* w, const int* hgt, const int* pitch, void* const* flow) {
    if (!h) return dis_fail(nullptr, DIS_EINVAL, "handle is NULL");
    if (n < 1 || !I0 || !I1 || !w || !hgt || !pitch || !flow)
        return dis_fail(h, DIS_EINVAL, "batch of %d pairs: NULL array or n < 1", n);
    if (n > h->max_batch) return dis_fail(h, DIS_ESIZE, "batch of %d pairs exceeds max_batch %d", n, h->max_batch);
    if (h->p.flags & (DIS_FLAG_FB_CONSISTENCY | DIS_FLAG_COLOUR))
        return dis_fail(h, DIS_EINVAL, "forward-backward consistency and colour frames run through dis_compute_flow only");
    for (int k = 0; k < n; ++k) {
        if (!I0[k] || !I1[k] || !flow[k]) return dis_fail(h, DIS_EINVAL, "pair %d: NULL frame or flow pointer", k);
        if (w[k] < 1 || hgt[k] < 1) return dis_fail(h, DIS_EINVAL, "pair %d: size %dx%d invalid", k, w[k], hgt[k]);
        if (pitch[k] < w[k]) return dis_fail(h, DIS_EINVAL, "pair %d: pitch %d < width %d", k, pitch[k], w[k]);
        if (w[k] > h->max_w || hgt[k] > h->max_h)
            return dis_fail(h, DIS_ESIZE, "pair %d: %dx%d exceeds the handle's %dx%d", k, w[k], hgt[k], h->max_w,
                            h->max_h);
    }
    std::vector<int> key;
    key.push_back(n);
    for (int k = 0; k < n; ++k) { key.push_back(w[k]); key.push_back(hgt[k]); key.push_back(pitch[k]); }
    BatchPlan* bp;
    auto it = h->bplans.find(key);
    if (it == h->bplans.end()) {
        bp = new BatchPlan();
        int r = build_batch(h, n, w, hgt, pitch, bp);
        if (r != DIS_OK) {
            dis_batch_plan_free(bp);
            return r;
        }
        h->bplans[key] = bp;
    } else {
        bp = it->second;
    }
    // upload new frame / flow pointers (only when they change)
    bool changed = false;
    for (int k = 0; k < n; ++k)
        if (bp->bound[3 * k] != I0[k] || bp->bound[3 * k + 1] != I1[k] || bp->bound[3 * k + 2] != flow[k]) changed = true;
    if (changed) {
        XHIPCHK(h, hipStreamSynchronize(h->stream));   // no earlier replay may still read the tables
        for (int k = 0; k < n; ++k) {
            bp->pyr0[k].src[0] = I0[k];
            bp->pyr0[k].src[1] = I1[k];
            bp->ups[k].out = flow[k];
            bp->bound[3 * k] = I0[k];
            bp->bound[3 * k + 1] = I1[k];
            bp->bound[3 * k + 2] = flow[k];
        }
        XHIPCHK(h, hipMemcpy((char*)bp->io + bp->pyr0_off, bp->pyr0.data(), sizeof(PyrArgs) * n,
                             hipMemcpyHostToDevice));
        XHIPCHK(h, hipMemcpy((char*)bp->io + bp->ups_off, bp->ups.data(), sizeof(UpsArgs) * n,
                             hipMemcpyHostToDevice));
    }
    int r;
    if ((h->p.flags & DIS_FLAG_NO_GRAPH) || h->profiling) {
        r = dis_launch_eager(h, bp->seq);
        if (r != DIS_OK) return r;
    } else {
        if (!bp->exec) {
            r = build_batch_graph(h, bp);
            if (r != DIS_OK) return r;
        }
        XHIPCHK(h, hipGraphLaunch(bp->exec, h->stream));
    }
    h->have_last = true;
    h->last_w = w[0];
    h->last_h = hgt[0];
    h->last_ss = bp->ss[0];
    h->last_sf = h->p.finest_scale;
    h->last_tabs = &bp->tabs;
    h->last_call = 2;
    h->last_batch.assign(I0, I0 + n);
    h->last_batch_I1.assign(I1, I1 + n);
    h->last_batch_flow.assign(flow, flow + n);
    h->last_batch_w.assign(w, w + n);
    h->last_batch_h.assign(hgt, hgt + n);
    h->last_batch_pitch.assign(pitch, pitch + n);
    return DIS_OK;
}

// ---------------------------------------------------------------- autotune

// Replay the most recent forward call under every launch choice that cannot
// change the result, keep the fastest, and append it to a JSON-lines file.
extern "C" int dis_autotune(dis_handle* h, const char* cache_path) {
    if (!h) return dis_fail(nullptr, DIS_EINVAL, "handle is NULL");
    if (h->last_call == 0) return dis_fail(h, DIS_ESTATE, "autotune replays the last forward call: none yet");
    struct Cand { int lpp, tile, mode; };
    // the search's lanes per patch and the refinement tile touch different
    // kernels of a phase-major launch, so they are tuned one after the other;
    // the persistent launch is tried with every lane count on each of its
    // two refinement tiles
    const int lpps[7] = {1, 2, 4, 8, 16, 32, 64};
    const int save_flags = (int)h->p.flags;
    h->p.flags &= ~DIS_FLAG_NO_GRAPH;   // time what callers run: graph replay
    auto replay = [&]() -> int {
        if (h->last_call == 1)
            return dis_compute_flow(h, h->last_I0, h->last_I1, h->last_w, h->last_h, h->last_pitch, h->last_flow);
        return dis_compute_flow_batched(h, (int)h->last_batch.size(), h->last_batch.data(), h->last_batch_I1.data(),
                                        h->last_batch_w.data(), h->last_batch_h.data(), h->last_batch_pitch.data(),
                                        h->last_batch_flow.data());
    };
    // copies: the replays overwrite the "last call" record
    const int call = h->last_call;
    const void *I0 = h->last_I0, *I1 = h->last_I1;
    void* flow = h->last_flow;
    const int lw = h->last_w, lh = h->last_h, lp = h->last_pitch;
    std::vector<const void*> b0 = h->last_batch, b1 = h->last_batch_I1;
    std::vector<void*> bf = h->last_batch_flow;
    std::vector<int> bw = h->last_batch_w, bh = h->last_batch_h, bpch = h->last_batch_pitch;
    auto restore = [&]() {
        h->last_call = call; h->last_I0 = I0; h->last_I1 = I1; h->last_flow = flow;
        h->last_w = lw; h->last_h = lh; h->last_pitch = lp;
        h->last_batch = b0; h->last_batch_I1 = b1; h->last_batch_flow = bf;
        h->last_batch_w = bw; h->last_batch_h = bh; h->last_batch_pitch = bpch;
    };
    // The replays read the last call's frames (which the caller keeps alive
    // and unchanged) but write their flow into buffers of their own: the
    // caller's flow buffers are never touched.
    const size_t elem = (h->p.flags & DIS_FLAG_IO_F64) ? sizeof(double) : sizeof(float);
    std::vector<void*> tmp_flow;
    auto free_tmp = [&]() {
        hipStreamSynchronize(h->stream);
        for (void* q : tmp_flow) hipFree(q);
        tmp_flow.clear();
    };
    {
        const int np = call == 1 ? 1 : (int)b0.size();
        for (int k = 0; k < np; ++k) {
            const size_t px = call == 1 ? (size_t)lw * lh : (size_t)bw[k] * bh[k];
            void* q = nullptr;
            if (hipMalloc(&q, 2 * px * elem) != hipSuccess) {
                free_tmp();
                return dis_fail(h, DIS_ENOMEM, "autotune: no memory for a %zu-pixel flow buffer", px);
            }
            tmp_flow.push_back(q);
        }
    }
    void* flow_tmp = call == 1 ? tmp_flow[0] : nullptr;
    std::vector<void*> bf_tmp = call == 1 ? std::vector<void*>() : tmp_flow;
    auto restore_tmp = [&]() {
        restore();
        h->last_flow = flow_tmp;
        h->last_batch_flow = bf_tmp;
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        free_tmp();
        return dis_fail(h, DIS_EHIP, "autotune: hipEventCreate failed");
    }
    double best = 1e30;
    Cand bestc{0, 0, 1};
    int best_lv[DIS_MAXL] = {0};   // lanes per patch of each scale in the best choice
    int r = DIS_OK;
    // times one choice; `lv` (per scale) overrides c.lpp
    auto measure = [&](const Cand& c, const int* lv_in = nullptr) -> int {
        int lv[DIS_MAXL];
        for (int s = 0; s < DIS_MAXL; ++s) lv[s] = lv_in ? lv_in[s] : c.lpp;
        int rr = dis_set_tunables(h, lv, c.tile, c.mode);
        if (rr != DIS_OK) return rr;
        for (int i = 0; i < 3 && rr == DIS_OK; ++i) { restore_tmp(); rr = replay(); }
        if (rr != DIS_OK) return rr;
        const int reps = 10;
        hipEventRecord(e0, h->stream);
        for (int i = 0; i < reps && rr == DIS_OK; ++i) { restore_tmp(); rr = replay(); }
        hipEventRecord(e1, h->stream);
        if (rr != DIS_OK) return rr;
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms / reps < best) {
            best = ms / reps;
            bestc = c;
            for (int s = 0; s < DIS_MAXL; ++s) best_lv[s] = lv[s];
        }
        return DIS_OK;
    };
    for (int t = 0; t < DIS_NUM_TILES && r == DIS_OK; ++t) r = measure(Cand{0, t, 1});
    const int tile = bestc.tile;
    for (int l : lpps)
        if (r == DIS_OK && dis_search_has_lanes(&h->p, l)) r = measure(Cand{l, tile, 1});
    if (r == DIS_OK) r = measure(Cand{bestc.lpp, bestc.tile, 3});    // single-workgroup scales of <= 256 pairs
    if (r == DIS_OK) r = measure(Cand{bestc.lpp, bestc.tile, 19});   // ... of <= 1024 pairs
    if (r == DIS_OK) r = measure(Cand{bestc.lpp, bestc.tile, bestc.mode | 8});   // no linearisation cache
    // the lean twin on the large scales (a tile that is lean itself has no other)
    const int twin = dis_refine_tile_lean(bestc.tile);
    if (r == DIS_OK && twin >= 0 && twin != bestc.tile && !(bestc.mode & 64))
        r = measure(Cand{bestc.lpp, bestc.tile, bestc.mode | 64});
    // the persistent launch, with each lane count, on its 32x16 tile and (row-owned search) its 16x16 one
    const bool rows = dis_search_rows_path(&h->p) && dis_channels(&h->p) == 1;
    for (int tile : {0, 1}) {
        if (tile == 1 && !rows) break;
        if (r == DIS_OK) r = measure(Cand{0, tile, 0});
        for (int l : lpps)
            if (r == DIS_OK && dis_search_has_lanes(&h->p, l) &&
                (rows ? dis_kernel_level_rows(h->p.patch_size, l, tile) : dis_kernel_level(h->p.patch_size, l)))
                r = measure(Cand{l, tile, 0});
    }
    // then the lanes per patch of each processed scale on its own (the scales'
    // searches differ in patch count), coarsest first, the others held
    {
        int top = dis_coarsest(&h->p, lw, lh);
        if (call != 1) {
            top = h->p.finest_scale;
            for (size_t k = 0; k < bw.size(); ++k) top = std::max(top, dis_coarsest(&h->p, bw[k], bh[k]));
        }
        const Cand c = bestc;
        for (int s = top; s >= h->p.finest_scale && r == DIS_OK; --s) {
            int cur[DIS_MAXL];
            std::memcpy(cur, best_lv, sizeof cur);
            for (int l : lpps) {
                if (r != DIS_OK || l == cur[s] || !dis_search_has_lanes(&h->p, l)) continue;
                if (!(c.mode & 1)) {   // the persistent launch has its own kernels per lane count
                    const bool ok = dis_search_rows_path(&h->p) && dis_channels(&h->p) == 1
                                        ? dis_kernel_level_rows(h->p.patch_size, l, dis_level_tile(c.tile, true)) != nullptr
                                        : dis_kernel_level(h->p.patch_size, l) != nullptr;
                    if (!ok) continue;
                }
                int t[DIS_MAXL];
                std::memcpy(t, cur, sizeof t);
                t[s] = l;
                r = measure(c, t);
            }
        }
    }
    free_tmp();
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    h->p.flags = (uint32_t)save_flags;
    restore();
    if (r != DIS_OK) return r;
    r = dis_set_tunables(h, best_lv, bestc.tile, bestc.mode);
    if (r != DIS_OK) return r;
    h->tuned_ms = best;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return dis_fail(h, DIS_EINVAL, "cannot open %s", cache_path);
        std::fprintf(f,
                     "{\"arch\": \"gfx950\", \"call\": \"%s\", \"w\": %d, \"h\": %d, \"pairs\": %d, \"patch\": %d, "
                     "\"overlap\": %g, \"iters\": %d, \"lanes_per_patch\": [",
                     call == 1 ? "plain" : "batched", lw, lh, call == 1 ? 1 : (int)b0.size(), h->p.patch_size,
                     h->p.overlap, h->p.gn_iters);
        for (int s = 0; s < DIS_MAXL; ++s) std::fprintf(f, "%s%d", s ? ", " : "", best_lv[s]);
        std::fprintf(f, "], \"refine_tile\": %d, \"launch_mode\": %d, \"ms\": %.5f}\n", bestc.tile, bestc.mode, best);
        std::fclose(f);
    }
    return DIS_OK;
}

