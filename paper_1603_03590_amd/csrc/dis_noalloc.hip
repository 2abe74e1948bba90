// dis_compute_flow_noalloc: the plain flow call for callers that cannot
// allocate device memory.  Its buffers live in one file-scope device array,
// so the call itself allocates nothing on the device.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "dis.h"
#include "dis_host.h"
#include "dis_internal.h"

// Every device this library runs on holds one copy of this array until the
// process ends.  Host code must never pass its name to a kernel or a copy:
// on the host the name stands for a host-side shadow, not the device copy.
static __device__ __align__(256) unsigned char scratch[DIS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

// One per device: the device address of `scratch`, and a host-side handle
// whose buffers sit inside it, with the launch sequence of the last frame
// size (the buffer offsets only depend on the parameters and the size).
struct DeviceState {
    char* ptr = nullptr;
    dis_handle* h = nullptr;
    Seq seq;
    bool have_seq = false;
    dis_params key_p{};
    int key_w = 0, key_h = 0, key_pitch = 0;
};

std::mutex g_mu;
DeviceState g_dev[kMaxDevices];

bool same_params(const dis_params& a, const dis_params& b) { return std::memcmp(&a, &b, sizeof a) == 0; }

// Fresh host handle for frames of w x hgt: default launch choices except
// that the refinement recomputes its linearisation (no cache buffer), and
// every buffer carved from the device's scratch.
int make_handle(DeviceState& d, const dis_params* p, int w, int hgt, int device, dis_handle** out) {
    dis_handle* h = new dis_handle();
    h->p = *p;
    h->max_w = w;
    h->max_h = hgt;
    h->max_batch = 1;
    h->device = device;
    h->st = dis_stride(p);
    h->top = dis_top_level(p, w, hgt);
    for (int s = 0; s < DIS_MAXL; ++s) h->lpp[s] = 0;
    h->refine_tile = 10;      // 8x4 cores on 384 threads
    h->mode_phase = 1;
    h->small_levels = 1;      // scales of <= 256 pixel pairs in one block
    h->no_lin_cache = 1;
    h->arena = d.ptr;
    h->arena_cap = DIS_NOALLOC_SCRATCH_BYTES;
    h->arena_used = 0;
    h->slots.resize(1);
    const int r = dis_alloc_slot(h, h->slots[0]);
    if (r != DIS_OK) {
        dis_fail(nullptr, r, "%s", h->err.c_str());
        delete h;
        return r;
    }
    *out = h;
    return DIS_OK;
}

}  // namespace

extern "C" int dis_compute_flow_noalloc(const dis_params* p, const void* I0, const void* I1, int w, int hgt,
                                        int pitch, void* flow, void* hip_stream) {
    int r = dis_validate_params(p);
    if (r != DIS_OK) return r;
    if (!I0 || !I1 || !flow) return dis_fail(nullptr, DIS_EINVAL, "NULL frame or flow pointer");
    if (w < 1 || hgt < 1) return dis_fail(nullptr, DIS_EINVAL, "size %dx%d invalid", w, hgt);
    if (pitch < w) return dis_fail(nullptr, DIS_EINVAL, "pitch %d < width %d", pitch, w);
    if (p->flags & (DIS_FLAG_KEEP_FOR_BACKWARD | DIS_FLAG_FB_CONSISTENCY | DIS_FLAG_COLOUR))
        return dis_fail(nullptr, DIS_EINVAL,
                        "the static-scratch call takes neither DIS_FLAG_KEEP_FOR_BACKWARD, "
                        "DIS_FLAG_FB_CONSISTENCY nor DIS_FLAG_COLOUR");
    if (w > 65536 || hgt > 65536) return dis_fail(nullptr, DIS_ESIZE, "size %dx%d too large", w, hgt);
    if ((w >> p->finest_scale) < p->patch_size || (hgt >> p->finest_scale) < p->patch_size)
        return dis_fail(nullptr, DIS_ESIZE, "%dx%d at scale %d is smaller than the %d px patch", w, hgt,
                        p->finest_scale, p->patch_size);
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return dis_fail(nullptr, DIS_EHIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (device < 0 || device >= kMaxDevices)
        return dis_fail(nullptr, DIS_EINVAL, "device %d beyond the %d this call serves", device, kMaxDevices);

    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState& d = g_dev[device];
    if (!d.ptr) {
        // first call on this device (current here): the device copy's address
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return dis_fail(nullptr, DIS_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        d.ptr = (char*)ptr;
    }
    if (!d.have_seq || d.key_w != w || d.key_h != hgt || d.key_pitch != pitch || !same_params(d.key_p, *p)) {
        d.have_seq = false;
        d.seq.items.clear();
        if (d.h) {
            delete d.h;
            d.h = nullptr;
        }
        dis_handle* h = nullptr;
        r = make_handle(d, p, w, hgt, device, &h);
        if (r != DIS_OK) return r;
        PlanTables tabs;
        PairInfo info{};
        r = dis_build_pair(h, h->slots[0], w, hgt, pitch, I0, I1, flow, d.seq, &info, tabs);
        if (r != DIS_OK) {
            dis_fail(nullptr, r, "%s", h->err.c_str());
            delete h;
            d.seq.items.clear();
            return r;
        }
        d.h = h;
        d.have_seq = true;
        d.key_p = *p;
        d.key_w = w;
        d.key_h = hgt;
        d.key_pitch = pitch;
    }
    // the caller's frames and flow for this call
    for (Launch& L : d.seq.items) {
        if (L.kind == 1) {
            PyrArgs* pa = (PyrArgs*)L.arg.data();
            pa->src[0] = I0;
            pa->src[1] = I1;
        } else if (L.kind == 2) {
            ((UpsArgs*)L.arg.data())->out = flow;
        }
    }
    d.h->stream = (hipStream_t)hip_stream;
    r = dis_launch_eager(d.h, d.seq);
    if (r != DIS_OK) return dis_fail(nullptr, r, "%s", d.h->err.c_str());
    return DIS_OK;
}
