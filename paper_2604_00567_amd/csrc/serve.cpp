// Serving slots: one in-flight launch of the persistent batch kernels over the
// requests admitted in one scheduling step.  The work list is built on the
// host, packed with the transform offsets into one pinned staging buffer and
// copied to the slot's device buffer with one copy on the slot's stream, so
// a step costs one copy and one launch per phase, and consecutive steps on
// different slots overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "batch_launch.hpp"
#include "dsfft.h"
#include "plan.hpp"
#include "tables.hpp"

struct fft_serve_slot {
    int dtype = 0, kind = 0, device = 0;
    std::shared_ptr<dsfft::DeviceTable> table;
    uint8_t* d_stage = nullptr;              // items, then the offsets
    unsigned* d_ctl = nullptr;
    void* ws = nullptr;
    uint8_t* h_stage = nullptr;              // pinned staging of the same layout
    int64_t item_cap = 0, offs_cap = 0;
    int slot_cap = 0;
    size_t ws_cap = 0;
    int resident = 1;
    int cfg_choice[17] = {};
    hipEvent_t done = nullptr;
    bool launched = false;
    std::vector<int64_t> tn, toff, offs, lists;
    int64_t nlist[dsfft::kNumLists] = {};
    std::vector<dsfft::HostBatchItem> items;
    ~fft_serve_slot();
};

fft_serve_slot::~fft_serve_slot() {
    if (done) {
        if (launched) (void)hipEventSynchronize(done);
        (void)hipEventDestroy(done);
    }
    if (d_stage) (void)hipFree(d_stage);
    if (d_ctl) (void)hipFree(d_ctl);
    if (ws) (void)hipFree(ws);
    if (h_stage) (void)hipHostFree(h_stage);
}

using namespace dsfft;

extern "C" {

fft_serve_slot* fft_serve_slot_create(fft_dtype dtype, fft_table_kind kind, int64_t max_items,
                                      int64_t max_transforms, int max_large, size_t ws_bytes) {
    if ((int)dtype != DT_F16 && (int)dtype != DT_F32) {
        set_error(FFT_EINVAL, "dtype must be FFT_F16 or FFT_F32");
        return nullptr;
    }
    if ((int)kind < 0 || (int)kind > 3 || max_items < 1 || max_transforms < 1 || max_large < 0) {
        set_error(FFT_EINVAL, "bad serving slot parameters");
        return nullptr;
    }
    std::unique_ptr<fft_serve_slot> s(new fft_serve_slot());
    s->dtype = (int)dtype;
    s->kind = (int)kind;
    s->item_cap = max_items;
    s->offs_cap = max_transforms;
    s->slot_cap = max_large;
    s->ws_cap = ws_bytes;
    for (int m = 1; m <= kMaxSingleLog; ++m) s->cfg_choice[m] = kSmallCfg[m];
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) { hip_error(e, "hipGetDevice"); return nullptr; }
    if (get_table(int64_t(1) << 18, s->dtype, s->kind, false, &s->table) != FFT_OK) return nullptr;
    const size_t stage = sizeof(HostBatchItem) * max_items + sizeof(int64_t) * max_transforms;
    if ((e = hipMalloc(&s->d_stage, stage)) != hipSuccess ||
        (e = hipMalloc(&s->d_ctl, sizeof(unsigned) * kQueueWords)) != hipSuccess ||
        (ws_bytes && (e = hipMalloc(&s->ws, ws_bytes)) != hipSuccess) ||
        (e = hipHostMalloc((void**)&s->h_stage, stage, 0)) != hipSuccess) {
        set_error(e == hipErrorOutOfMemory ? FFT_ENOMEM : FFT_EHIP, "serving slot allocation failed");
        return nullptr;
    }
    if ((e = hipMemset(s->d_ctl, 0, sizeof(unsigned) * kQueueWords)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess) {
        hip_error(e, "hipMemset(queue words)");
        return nullptr;
    }
    if (batch_resident_grid(s->dtype, s->device, &s->resident) != FFT_OK) return nullptr;
    if ((e = hipEventCreateWithFlags(&s->done, hipEventDisableTiming)) != hipSuccess) {
        hip_error(e, "hipEventCreate");
        return nullptr;
    }
    return s.release();
}

// Launches requests r = 0..nreq-1: batch[r] transforms of n[r] points each,
// in place at element offsets off[r] + j * n[r] of `data`.  Waits first for
// the slot's previous launch (its staging buffers are reused).
int fft_serve_slot_launch(fft_serve_slot* s, const int64_t* n, const int64_t* batch,
                          const int64_t* off, int64_t nreq, void* data, void* stream) {
    if (!s || !n || !batch || !off || nreq < 0) return set_error(FFT_EINVAL, "null argument");
    if (!data) return set_error(FFT_EINVAL, "null data pointer");
    if ((uintptr_t)data % (uintptr_t)elem_bytes(s->dtype))
        return set_error(FFT_EINVAL, "data must be aligned to the element size");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (s->launched && (e = hipEventSynchronize(s->done)) != hipSuccess)
        return hip_error(e, "hipEventSynchronize");
    s->tn.clear();
    s->toff.clear();
    int64_t nlarge = 0;
    for (int64_t r = 0; r < nreq; ++r) {
        const int64_t v = n[r];
        if (v < 2 || (v & (v - 1)) || v > (int64_t(1) << 18) || batch[r] < 1 || off[r] < 0)
            return set_error(FFT_EINVAL, "request sizes must be powers of two in [2, 2^18]");
        for (int64_t j = 0; j < batch[r]; ++j) {
            s->tn.push_back(v);
            s->toff.push_back(off[r] + j * v);
        }
        if (v > (int64_t(1) << max_whole_log(s->dtype))) nlarge += batch[r];
    }
    int64_t ws_elems = 0, phase0 = 0;
    build_work(s->tn.data(), s->toff.data(), (int64_t)s->tn.size(), s->cfg_choice,
               lists_for(s->dtype), s->items, s->offs, s->lists, s->nlist, ws_elems, phase0);
    if ((int64_t)s->items.size() > s->item_cap ||
        (int64_t)(s->offs.size() + s->lists.size()) > s->offs_cap || nlarge > s->slot_cap ||
        (size_t)ws_elems * elem_bytes(s->dtype) > s->ws_cap)
        return set_error(FFT_ENOMEM, "step exceeds the slot's capacity");
    if (s->items.empty() && s->lists.empty()) return FFT_OK;
    // staging layout: work items, single-unit offsets, list-kernel offsets
    const size_t ib = sizeof(HostBatchItem) * s->items.size();   // a multiple of 8
    const size_t ob = sizeof(int64_t) * s->offs.size();
    const size_t bb = sizeof(int64_t) * s->lists.size();
    std::memcpy(s->h_stage, s->items.data(), ib);
    std::memcpy(s->h_stage + ib, s->offs.data(), ob);
    std::memcpy(s->h_stage + ib + ob, s->lists.data(), bb);
    if ((e = hipMemcpyAsync(s->d_stage, s->h_stage, ib + ob + bb, hipMemcpyHostToDevice, st)) !=
        hipSuccess)
        return hip_error(e, "hipMemcpyAsync(work list)");
    const int64_t* d_lists = (const int64_t*)(s->d_stage + ib + ob);
    for (int i = 0; i < kNumLists; ++i) {
        if (s->nlist[i] && (e = launch_batch_list(i, data, data, s->table->ptr, d_lists, s->nlist[i], st)) !=
                               hipSuccess)
            return hip_error(e, "launch(list)");
        d_lists += s->nlist[i];
    }
    const int64_t n1 = (int64_t)s->items.size() - phase0;
    const int grid0 = (int)std::max<int64_t>(1, std::min<int64_t>(phase0, s->resident));
    const int grid1 = (int)std::max<int64_t>(1, std::min<int64_t>(n1, s->resident));
    if ((e = launch_batch_phases(s->dtype, data, data, s->ws, s->table->ptr, s->d_stage,
                                 (const int64_t*)(s->d_stage + ib),
                                 (int)phase0, (int)s->items.size(), s->d_ctl, grid0, grid1, st)) !=
        hipSuccess)
        return hip_error(e, "launch(batch)");
    if ((e = hipEventRecord(s->done, st)) != hipSuccess) return hip_error(e, "hipEventRecord");
    s->launched = true;
    return FFT_OK;
}

// 1 if the slot's last launch has finished (or none was made), 0 if running.
int fft_serve_slot_query(fft_serve_slot* s) {
    if (!s) return set_error(FFT_EINVAL, "null slot");
    if (!s->launched) return 1;
    hipError_t e = hipEventQuery(s->done);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return hip_error(e, "hipEventQuery");
}

void fft_serve_slot_destroy(fft_serve_slot* s) { delete s; }

}  // extern "C"
