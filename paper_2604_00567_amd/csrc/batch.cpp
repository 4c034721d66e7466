// Uneven-size batch plans: work-item construction, the HIP graph of the two
// persistent-kernel phases (fft_batch.hpp) and its replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "batch_launch.hpp"
#include "dsfft.h"
#include "plan.hpp"
#include "tables.hpp"

namespace dsfft {

// Single-unit configuration per log2 N (1..13) and units per workgroup.
const int kSmallCfg[kMaxSingleLog + 1] = {-1, HB_N2, HB_N4, HB_N8, HB_N16, HB_N32, HB_N64, HB_N128,
                                          HB_N256, HB_N512, HB_N1024, HB_N2048, HB_N4096, HB_N8192,
                                          HB_N16384};
const int kAltCfg[kMaxSingleLog + 1] = {-1, -1, -1, -1, -1, -1, -1, HB_N128_B, HB_N256_B, HB_N512_B,
                                        HB_N1024_B, HB_N2048_B, HB_N4096_B, -1, -1};
int cfg_upw(int cfg) {
    switch (cfg) {
        case HB_N2: case HB_N4: case HB_N8: return 512;
        case HB_N16: case HB_N32: return 128;
        case HB_N64: case HB_N128: case HB_ROWS128: case HB_COLS256:
        case HB_ROWS256: return 64;
        case HB_N256: case HB_N512: case HB_COLS512: case HB_ROWS512: case HB_N128_B: return 32;
        case HB_N1024: case HB_N256_B: case HB_N512_B: return 16;
        case HB_N2048: case HB_N1024_B: return 8;
        case HB_N4096_B: case HB_N2048_B: return 4;
        case HB_N16384: return 1;
        default: return 2;       // HB_N4096, HB_N8192
    }
}

}  // namespace dsfft

struct fft_batch {
    int dtype = 0, kind = 0, device = 0;
    int64_t count = 0, total = 0;
    std::vector<int64_t> n, offset;
    int cfg_choice[17] = {};                 // per log2 N (single-unit sizes)
    std::shared_ptr<dsfft::DeviceTable> table;
    std::vector<dsfft::HostBatchItem> items;
    std::vector<int64_t> offs, lists;        // lists: offsets for the list kernels
    int64_t nlist[dsfft::kNumLists] = {};
    dsfft::HostBatchItem* d_items = nullptr;
    int64_t* d_lists = nullptr;
    int64_t* d_offs = nullptr;
    unsigned* d_ctl = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int64_t phase0 = 0;                    // items of phase 0 (the rest are phase 1)
    int grid = 0, grid0 = 0, grid1 = 0, resident = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t knode[2] = {nullptr, nullptr};
    hipGraphNode_t lnode[dsfft::kNumLists] = {};   // list kernels (binary16 2^16, 2^15)
    const void* cap_in = nullptr;
    void* cap_out = nullptr;
    ~fft_batch();
};

// The batch's launches may still use its buffers: free them once the device
// has finished the work enqueued so far (an event per execute would cost
// device time on every replay).
fft_batch::~fft_batch() {
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    if (have_cur && cur != device) (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_items) (void)hipFree(d_items);
    if (d_offs) (void)hipFree(d_offs);
    if (d_lists) (void)hipFree(d_lists);
    if (d_ctl) (void)hipFree(d_ctl);
    if (ws) (void)hipFree(ws);
    if (have_cur && cur != device) (void)hipSetDevice(cur);
}

namespace dsfft {

// Column/row split of a transform of 2^15 .. 2^18 points (smaller ones are
// whole-transform items): configurations and log2 of the column count
// (column kernel) and row count (row kernel).
struct Split {
    int ccfg, rcfg, lm_c, lm_r;
};
static Split split_for(int m) {
    switch (m) {
        case 15: return {HB_COLS256, HB_ROWS128, 7, 8};
        case 16: return {HB_COLS256, HB_ROWS256, 8, 8};
        case 17: return {HB_COLS512, HB_ROWS256, 8, 9};
        default: return {HB_COLS512, HB_ROWS512, 9, 9};   // 18
    }
}

int64_t work_items_of_class(int dtype, int m, int64_t count) {
    if (count <= 0) return 0;
    if (m <= kMaxSingleLog) {
        const int64_t upw = cfg_upw(kSmallCfg[m]);
        return (count + upw - 1) / upw;
    }
    if (m <= max_whole_log(dtype)) return 0;      // list kernels
    const Split sp = split_for(m);
    const int64_t cu = cfg_upw(sp.ccfg), ru = cfg_upw(sp.rcfg);
    return count * (((int64_t(1) << sp.lm_c) + cu - 1) / cu + ((int64_t(1) << sp.lm_r) + ru - 1) / ru);
}

// Work items for transforms of sizes n[t] at element offsets off[t]:
// phase 0 = the column items of every large transform (in input order), then
// the single-unit items from the largest size down (so the end of the phase
// is made of short items); phase 1 = the row items.  Large transforms take
// consecutive workspace slices; ws_elems returns their total.
void build_work(const int64_t* n, const int64_t* off, int64_t count, const int* cfg_choice,
                int nlists, std::vector<HostBatchItem>& items, std::vector<int64_t>& offs,
                std::vector<int64_t>& lists, int64_t* nlist, int64_t& ws_elems, int64_t& phase0) {
    items.clear();
    offs.clear();
    lists.clear();
    std::vector<int64_t> per_list[kNumLists];
    std::vector<HostBatchItem> rows;
    std::vector<std::vector<int64_t>> by_class(19);
    ws_elems = 0;
    int slot = 0;
    for (int64_t t = 0; t < count; ++t) {
        int m = 0;
        while ((int64_t(1) << m) < n[t]) ++m;
        if (m <= kMaxSingleLog) {
            by_class[m].push_back(off[t]);
            continue;
        }
        int li = -1;
        for (int i = 0; i < nlists; ++i)
            if (m == kListLog[i]) li = i;
        if (li >= 0) {
            per_list[li].push_back(off[t]);
            continue;
        }
        const Split sp = split_for(m);
        const int cu = cfg_upw(sp.ccfg), ru = cfg_upw(sp.rcfg);
        const int ncols = 1 << sp.lm_c, nrows = 1 << sp.lm_r;
        for (int r0 = 0; r0 < ncols; r0 += cu) {
            HostBatchItem it{};
            it.cfg = sp.ccfg;
            it.nunits = std::min(cu, ncols - r0);
            it.first = r0;
            it.log_m = sp.lm_c;
            it.phase = 0;
            it.slot = slot;
            it.in_off = off[t];
            it.out_off = ws_elems;
            items.push_back(it);
        }
        for (int q0 = 0; q0 < nrows; q0 += ru) {
            HostBatchItem it{};
            it.cfg = sp.rcfg;
            it.nunits = std::min(ru, nrows - q0);
            it.first = q0;
            it.log_m = sp.lm_r;
            it.phase = 1;
            it.slot = slot;
            it.in_off = ws_elems;
            it.out_off = off[t];
            rows.push_back(it);
        }
        ws_elems += n[t];
        ++slot;
    }
    for (int m = kMaxSingleLog; m >= 1; --m) {
        const auto& v = by_class[m];
        if (v.empty()) continue;
        const int cfg = cfg_choice[m];
        const int upw = cfg_upw(cfg);
        for (size_t i = 0; i < v.size(); i += upw) {
            HostBatchItem it{};
            it.cfg = cfg;
            it.nunits = (int)std::min<size_t>(upw, v.size() - i);
            it.first = (int)offs.size();
            it.phase = 0;
            it.slot = -1;
            for (int k = 0; k < it.nunits; ++k) offs.push_back(v[i + k]);
            items.push_back(it);
        }
    }
    phase0 = (int64_t)items.size();
    items.insert(items.end(), rows.begin(), rows.end());
    for (int i = 0; i < kNumLists; ++i) {
        nlist[i] = (int64_t)per_list[i].size();
        lists.insert(lists.end(), per_list[i].begin(), per_list[i].end());
    }
}

static int build_items(fft_batch* b) {
    if (batch_resident_grid(b->dtype, b->device, &b->resident) != FFT_OK) return FFT_EHIP;
    int64_t ws_elems = 0;
    build_work(b->n.data(), b->offset.data(), b->count, b->cfg_choice, lists_for(b->dtype),
               b->items, b->offs, b->lists, b->nlist, ws_elems, b->phase0);
    b->ws_bytes = (size_t)ws_elems * elem_bytes(b->dtype);
    return FFT_OK;
}

// Resident workgroups of the persistent kernel (its grid when the work list is
// long enough).
int batch_resident_grid(int dtype, int device, int* out) {
    int cus = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return hip_error(e, "hipDeviceGetAttribute");
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel_func(dtype),
                                                     kHostBatchThreads, batch_lds_bytes(dtype));
    if (e != hipSuccess) return hip_error(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    *out = cus * std::max(per_cu, 1);
    return FFT_OK;
}

static int upload(fft_batch* b) {
    hipError_t e;
    if (b->d_items) { (void)hipFree(b->d_items); b->d_items = nullptr; }
    if (b->d_offs) { (void)hipFree(b->d_offs); b->d_offs = nullptr; }
    if (b->d_lists) { (void)hipFree(b->d_lists); b->d_lists = nullptr; }
    if (b->d_ctl) { (void)hipFree(b->d_ctl); b->d_ctl = nullptr; }
    if (b->ws) { (void)hipFree(b->ws); b->ws = nullptr; }
    const size_t ib = std::max<size_t>(1, b->items.size()) * sizeof(HostBatchItem);
    const size_t ob = std::max<size_t>(1, b->offs.size()) * sizeof(int64_t);
    if ((e = hipMalloc(&b->d_items, ib)) != hipSuccess) return hip_error(e, "hipMalloc(items)");
    if ((e = hipMalloc(&b->d_offs, ob)) != hipSuccess) return hip_error(e, "hipMalloc(offsets)");
    if (!b->lists.empty() &&
        (e = hipMalloc(&b->d_lists, b->lists.size() * sizeof(int64_t))) != hipSuccess)
        return hip_error(e, "hipMalloc(list offsets)");
    if ((e = hipMalloc(&b->d_ctl, sizeof(unsigned) * kQueueWords)) != hipSuccess)
        return hip_error(e, "hipMalloc(control)");
    if (b->ws_bytes && (e = hipMalloc(&b->ws, b->ws_bytes)) != hipSuccess)
        return e == hipErrorOutOfMemory ? set_error(FFT_ENOMEM, "batch workspace allocation failed")
                                        : hip_error(e, "hipMalloc(workspace)");
    if (!b->items.empty() &&
        (e = hipMemcpy(b->d_items, b->items.data(), b->items.size() * sizeof(HostBatchItem),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return hip_error(e, "hipMemcpy(items)");
    if (!b->offs.empty() &&
        (e = hipMemcpy(b->d_offs, b->offs.data(), b->offs.size() * sizeof(int64_t),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return hip_error(e, "hipMemcpy(offsets)");
    if (!b->lists.empty() &&
        (e = hipMemcpy(b->d_lists, b->lists.data(), b->lists.size() * sizeof(int64_t),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return hip_error(e, "hipMemcpy(list offsets)");
    if ((e = hipMemset(b->d_ctl, 0, sizeof(unsigned) * kQueueWords)) != hipSuccess)
        return hip_error(e, "hipMemset(queue words)");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_error(e, "hipDeviceSynchronize");
    const int64_t n1 = (int64_t)b->items.size() - b->phase0;
    b->grid0 = (int)std::max<int64_t>(1, std::min<int64_t>(b->phase0, b->resident));
    b->grid1 = (int)std::max<int64_t>(1, std::min<int64_t>(n1, b->resident));
    b->grid = std::max(b->grid0, b->grid1);
    return FFT_OK;
}

// Kernel-node arguments of one phase; the pointers in `slots` must outlive
// the hipGraphAddKernelNode / hipGraphExecKernelNodeSetParams call.
struct PhaseArgs {
    const void* in;
    void* out;
    void* ws;
    const void* lt;
    const void* items;
    const int64_t* offs;
    int first, nitems;
    unsigned* head;
    void* slots[9];
    PhaseArgs(const fft_batch* b, const void* in_, void* out_, int phase)
        : in(in_), out(out_), ws(b->ws), lt(b->table->ptr), items(b->d_items), offs(b->d_offs),
          first(phase == 0 ? 0 : (int)b->phase0),
          nitems(phase == 0 ? (int)b->phase0 : (int)((int64_t)b->items.size() - b->phase0)),
          head(b->d_ctl + 2 * phase) {
        void* p[9] = {&in, &out, &ws, &lt, &items, &offs, &first, &nitems, &head};
        std::copy(p, p + 9, slots);
    }
};

static hipKernelNodeParams phase_params(const fft_batch* b, PhaseArgs& a, int phase) {
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(batch_kernel_func(b->dtype));
    kp.gridDim = dim3(phase == 0 ? b->grid0 : b->grid1);
    kp.blockDim = dim3(kHostBatchThreads);
    kp.sharedMemBytes = (unsigned)batch_lds_bytes(b->dtype);
    kp.kernelParams = a.slots;
    kp.extra = nullptr;
    return kp;
}

// Kernel-node arguments of list kernel `list`.
struct ListArgs {
    const void* in;
    void* out;
    const void* lt;
    const int64_t* offs;
    int64_t count;
    void* slots[5];
    ListArgs(const fft_batch* b, const void* in_, void* out_, int list)
        : in(in_), out(out_), lt(b->table->ptr),
          offs(b->d_lists + (list == 0 ? 0 : b->nlist[0])), count(b->nlist[list]) {
        void* p[5] = {&in, &out, &lt, &offs, &count};
        std::copy(p, p + 5, slots);
    }
};

static hipKernelNodeParams list_params(const fft_batch* b, ListArgs& a, int list) {
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(batch_list_func(list));
    kp.gridDim = dim3((unsigned)b->nlist[list]);
    kp.blockDim = dim3(kListThreads);
    kp.sharedMemBytes = (unsigned)batch_list_lds_bytes(list);
    kp.kernelParams = a.slots;
    kp.extra = nullptr;
    return kp;
}

// Builds the graph once: the list kernels (those with transforms) and phase 0
// as independent roots (they touch disjoint transforms, so each can fill the
// others' tails), then phase 1 after phase 0 (each phase a persistent kernel
// whose workgroups only claim items from a queue, so sharing the device with
// the list kernels never blocks them).
static int build_graph(fft_batch* b, const void* in, void* out) {
    hipError_t e;
    if ((e = hipGraphCreate(&b->graph, 0)) != hipSuccess) return hip_error(e, "hipGraphCreate");
    for (int i = 0; i < kNumLists; ++i) {
        if (b->nlist[i] == 0) continue;
        ListArgs la(b, in, out, i);
        hipKernelNodeParams kp = list_params(b, la, i);
        if ((e = hipGraphAddKernelNode(&b->lnode[i], b->graph, nullptr, 0, &kp)) != hipSuccess)
            return hip_error(e, "hipGraphAddKernelNode(list)");
    }
    hipGraphNode_t prev = nullptr;
    for (int ph = 0; ph < 2; ++ph) {
        PhaseArgs a(b, in, out, ph);
        if (a.nitems == 0) continue;
        hipKernelNodeParams kp = phase_params(b, a, ph);
        if ((e = hipGraphAddKernelNode(&b->knode[ph], b->graph, prev ? &prev : nullptr, prev ? 1 : 0,
                                       &kp)) != hipSuccess)
            return hip_error(e, "hipGraphAddKernelNode(phase)");
        prev = b->knode[ph];
    }
    if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
        return hip_error(e, "hipGraphInstantiate");
    b->cap_in = in;
    b->cap_out = out;
    return FFT_OK;
}

// Points the kernel nodes at new data buffers.
static int retarget(fft_batch* b, const void* in, void* out) {
    for (int i = 0; i < kNumLists; ++i) {
        if (!b->lnode[i]) continue;
        ListArgs la(b, in, out, i);
        hipKernelNodeParams kp = list_params(b, la, i);
        hipError_t e = hipGraphExecKernelNodeSetParams(b->exec, b->lnode[i], &kp);
        if (e != hipSuccess) return hip_error(e, "hipGraphExecKernelNodeSetParams(list)");
    }
    for (int ph = 0; ph < 2; ++ph) {
        if (!b->knode[ph]) continue;
        PhaseArgs a(b, in, out, ph);
        hipKernelNodeParams kp = phase_params(b, a, ph);
        hipError_t e = hipGraphExecKernelNodeSetParams(b->exec, b->knode[ph], &kp);
        if (e != hipSuccess) return hip_error(e, "hipGraphExecKernelNodeSetParams");
    }
    b->cap_in = in;
    b->cap_out = out;
    return FFT_OK;
}

int batch_execute(fft_batch* b, const void* in, void* out, hipStream_t s) {
    if (!b) return set_error(FFT_EINVAL, "null batch");
    if (!in || !out) return set_error(FFT_EINVAL, "null data pointer");
    const size_t eb = (size_t)elem_bytes(b->dtype);
    if (((uintptr_t)in % eb) || ((uintptr_t)out % eb))
        return set_error(FFT_EINVAL, "data pointers must be aligned to the element size");
    const uintptr_t x = (uintptr_t)in, y = (uintptr_t)out;
    const size_t bytes = (size_t)b->total * eb;
    if (x != y && x < y + bytes && y < x + bytes)
        return set_error(FFT_EINVAL, "in and out partially overlap");
    if (b->items.empty() && b->lists.empty()) return FFT_OK;
    int rc = FFT_OK;
    if (!b->exec) rc = build_graph(b, in, out);
    else if (b->cap_in != in || b->cap_out != out) rc = retarget(b, in, out);
    if (rc != FFT_OK) return rc;
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
    return FFT_OK;
}

// alt: per log2 N (0 .. kMaxSingleLog), 1 to take kAltCfg instead of
// kSmallCfg (NULL: every class its default).
fft_batch* batch_create(const int64_t* n, int64_t count, int dtype, int kind, const int* alt) {
    if (!n || count < 1) {
        set_error(FFT_EINVAL, "need at least one transform");
        return nullptr;
    }
    if (dtype != DT_F16 && dtype != DT_F32) {
        set_error(FFT_EINVAL, "dtype must be FFT_F16 or FFT_F32");
        return nullptr;
    }
    if (kind < 0 || kind > 3) {
        set_error(FFT_EINVAL, "unknown table kind");
        return nullptr;
    }
    std::unique_ptr<fft_batch> b(new fft_batch());
    b->dtype = dtype;
    b->kind = kind;
    b->count = count;
    int64_t nmax = 2;
    for (int64_t i = 0; i < count; ++i) {
        const int64_t v = n[i];
        if (v < 2 || (v & (v - 1)) || v > (int64_t(1) << 18)) {
            set_error(FFT_EINVAL, "batch sizes must be powers of two in [2, 2^18]");
            return nullptr;
        }
        b->n.push_back(v);
        b->offset.push_back(b->total);
        b->total += v;
        nmax = std::max(nmax, v);
    }
    for (int m = 1; m <= kMaxSingleLog; ++m) b->cfg_choice[m] = kSmallCfg[m];
    if (alt)
        for (int m = 1; m <= kMaxSingleLog; ++m)
            if (alt[m] == 1 && kAltCfg[m] >= 0) b->cfg_choice[m] = kAltCfg[m];
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        hip_error(e, "hipGetDevice");
        return nullptr;
    }
    if (get_table(nmax, dtype, kind, false, &b->table) != FFT_OK) return nullptr;
    if (build_items(b.get()) != FFT_OK) return nullptr;
    if (upload(b.get()) != FFT_OK) return nullptr;
    return b.release();
}

}  // namespace dsfft

using namespace dsfft;

extern "C" {

fft_batch* fft_batch_create(const int64_t* n, int64_t count, fft_dtype dtype, fft_table_kind kind) {
    return batch_create(n, count, (int)dtype, (int)kind, nullptr);
}

fft_batch* fft_batch_create_tuned(const int64_t* n, int64_t count, fft_dtype dtype,
                                  fft_table_kind kind, int choice_1024, int choice_4096) {
    int alt[kMaxSingleLog + 1] = {};
    alt[10] = choice_1024 == 1;
    alt[12] = choice_4096 == 1;
    return batch_create(n, count, (int)dtype, (int)kind, alt);
}

fft_batch* fft_batch_create_classes(const int64_t* n, int64_t count, fft_dtype dtype,
                                    fft_table_kind kind, const int32_t* alt) {
    int a[kMaxSingleLog + 1] = {};
    if (alt)
        for (int m = 1; m <= kMaxSingleLog; ++m) a[m] = alt[m] == 1;
    return batch_create(n, count, (int)dtype, (int)kind, a);
}

int fft_batch_execute(fft_batch* b, const void* in, void* out, void* stream) {
    return batch_execute(b, in, out, (hipStream_t)stream);
}

int fft_batch_elements(const fft_batch* b, int64_t* elements) {
    if (!b || !elements) return set_error(FFT_EINVAL, "null argument");
    *elements = b->total;
    return FFT_OK;
}

int fft_batch_info(const fft_batch* b, int64_t* items, int64_t* grid, size_t* workspace_bytes) {
    if (!b) return set_error(FFT_EINVAL, "null batch");
    if (items) *items = (int64_t)b->items.size();
    if (grid) *grid = b->grid;
    if (workspace_bytes) *workspace_bytes = b->ws_bytes;
    return FFT_OK;
}

void fft_batch_destroy(fft_batch* b) { delete b; }

int fft_batch_work_list(const int64_t* n, int64_t count, fft_dtype dtype, int64_t* items_out,
                        int64_t item_cap, int64_t* nitems, int64_t* phase0, int64_t* offs_out,
                        int64_t offs_cap, int64_t* noffs, int64_t* list_out, int64_t list_cap,
                        int64_t* nlist, int64_t* ws_elems) {
    if (!n || count < 0 || !nitems || !phase0 || !noffs || !nlist || !ws_elems)
        return set_error(FFT_EINVAL, "null argument");
    if ((int)dtype != DT_F16 && (int)dtype != DT_F32) return set_error(FFT_EINVAL, "bad dtype");
    std::vector<int64_t> sizes(n, n + count), offset(count);
    int64_t total = 0;
    for (int64_t i = 0; i < count; ++i) {
        const int64_t v = n[i];
        if (v < 2 || (v & (v - 1)) || v > (int64_t(1) << 18))
            return set_error(FFT_EINVAL, "batch sizes must be powers of two in [2, 2^18]");
        offset[i] = total;
        total += v;
    }
    std::vector<HostBatchItem> items;
    std::vector<int64_t> offs, lists;
    int64_t per[kNumLists] = {};
    build_work(sizes.data(), offset.data(), count, kSmallCfg, lists_for((int)dtype), items, offs,
               lists, per, *ws_elems, *phase0);
    *nitems = (int64_t)items.size();
    *noffs = (int64_t)offs.size();
    *nlist = (int64_t)lists.size();
    if (!items_out && !offs_out && !list_out) return FFT_OK;     // size query
    if ((int64_t)items.size() > item_cap || (int64_t)offs.size() > offs_cap ||
        (int64_t)lists.size() > list_cap)
        return set_error(FFT_EINVAL, "output capacity too small (sizes returned in nitems, noffs, nlist)");
    for (size_t i = 0; i < items.size(); ++i) {
        const HostBatchItem& it = items[i];
        const int64_t row[8] = {it.cfg, it.nunits, it.first, it.log_m, it.phase, it.slot,
                                it.in_off, it.out_off};
        std::copy(row, row + 8, items_out + 8 * i);
    }
    std::copy(offs.begin(), offs.end(), offs_out);
    std::copy(lists.begin(), lists.end(), list_out);
    return FFT_OK;
}

}  // extern "C"
