// Uneven-size batch plans: work-item construction, HIP graph capture and
// replay of the persistent kernel (fft_batch.hpp), per-class tuning.
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
const int kSmallCfg[14] = {-1, HB_N2, HB_N4, HB_N8, HB_N16, HB_N32, HB_N64, HB_N128,
                                  HB_N256, HB_N512, HB_N1024, HB_N2048, HB_N4096, HB_N8192};
int cfg_upw(int cfg) {
    switch (cfg) {
        case HB_N2: case HB_N4: case HB_N8: return 256;
        case HB_N16: case HB_N32: return 64;
        case HB_N64: case HB_N128: case HB_COLS128: case HB_ROWS128: return 32;
        case HB_N256: case HB_N512: case HB_COLS256: case HB_ROWS256: case HB_COLS512:
        case HB_ROWS512: return 16;
        case HB_N1024: return 8;
        case HB_N2048: case HB_N1024_B: return 4;
        case HB_N4096_B: return 2;
        default: return 1;       // HB_N4096, HB_N8192
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
    std::vector<int64_t> offs;
    dsfft::HostBatchItem* d_items = nullptr;
    int64_t* d_offs = nullptr;
    unsigned* d_ctl = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int nslots = 0, ctl_words = 0, grid = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t knode = nullptr;
    const void* cap_in = nullptr;
    void* cap_out = nullptr;
    hipEvent_t last = nullptr;
    ~fft_batch();
};

fft_batch::~fft_batch() {
    if (last) {
        (void)hipEventSynchronize(last);
        (void)hipEventDestroy(last);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (d_items) (void)hipFree(d_items);
    if (d_offs) (void)hipFree(d_offs);
    if (d_ctl) (void)hipFree(d_ctl);
    if (ws) (void)hipFree(ws);
}

namespace dsfft {

// Column/row split of a large transform: configurations and log2 of the
// column count (column kernel) and row count (row kernel).
struct Split {
    int ccfg, rcfg, lm_c, lm_r;
};
static Split split_for(int m) {
    switch (m) {
        case 14: return {HB_COLS128, HB_ROWS128, 7, 7};
        case 15: return {HB_COLS256, HB_ROWS128, 7, 8};
        case 16: return {HB_COLS256, HB_ROWS256, 8, 8};
        case 17: return {HB_COLS512, HB_ROWS256, 8, 9};
        default: return {HB_COLS512, HB_ROWS512, 9, 9};   // 18
    }
}

// Work items for transforms of sizes n[t] at element offsets off[t]: column
// items of every large transform first, then single-unit items from the
// largest size down, then row items (which wait on their transform's column
// items, all queued earlier).  Large transforms take consecutive workspace
// slices; ws_elems returns their total, nslots the number of counters.
void build_work(const int64_t* n, const int64_t* off, int64_t count, const int* cfg_choice,
                std::vector<HostBatchItem>& items, std::vector<int64_t>& offs, int64_t& ws_elems,
                int& nslots) {
    items.clear();
    offs.clear();
    std::vector<HostBatchItem> cols, rows, small;
    std::vector<std::vector<int64_t>> by_class(19);
    ws_elems = 0;
    int slot = 0;
    for (int64_t t = 0; t < count; ++t) {
        int m = 0;
        while ((int64_t(1) << m) < n[t]) ++m;
        if (m <= 13) {
            by_class[m].push_back(off[t]);
            continue;
        }
        const Split sp = split_for(m);
        const int cu = cfg_upw(sp.ccfg), ru = cfg_upw(sp.rcfg);
        const int ncols = 1 << sp.lm_c, nrows = 1 << sp.lm_r;
        int citems = 0;
        for (int r0 = 0; r0 < ncols; r0 += cu, ++citems) {
            HostBatchItem it{};
            it.cfg = sp.ccfg;
            it.nunits = std::min(cu, ncols - r0);
            it.first = r0;
            it.log_m = sp.lm_c;
            it.wait_slot = -1;
            it.post_slot = slot;
            it.in_off = off[t];
            it.out_off = ws_elems;
            cols.push_back(it);
        }
        for (int q0 = 0; q0 < nrows; q0 += ru) {
            HostBatchItem it{};
            it.cfg = sp.rcfg;
            it.nunits = std::min(ru, nrows - q0);
            it.first = q0;
            it.log_m = sp.lm_r;
            it.wait_slot = slot;
            it.wait_need = citems;
            it.post_slot = -1;
            it.in_off = ws_elems;
            it.out_off = off[t];
            rows.push_back(it);
        }
        ws_elems += n[t];
        ++slot;
    }
    for (int m = 13; m >= 1; --m) {
        const auto& v = by_class[m];
        if (v.empty()) continue;
        const int cfg = cfg_choice[m];
        const int upw = cfg_upw(cfg);
        for (size_t i = 0; i < v.size(); i += upw) {
            HostBatchItem it{};
            it.cfg = cfg;
            it.nunits = (int)std::min<size_t>(upw, v.size() - i);
            it.first = (int)offs.size();
            it.wait_slot = -1;
            it.post_slot = -1;
            for (int k = 0; k < it.nunits; ++k) offs.push_back(v[i + k]);
            small.push_back(it);
        }
    }
    items = cols;
    items.insert(items.end(), small.begin(), small.end());
    items.insert(items.end(), rows.begin(), rows.end());
    nslots = slot;
}

static void build_items(fft_batch* b) {
    int64_t ws_elems = 0;
    build_work(b->n.data(), b->offset.data(), b->count, b->cfg_choice, b->items, b->offs, ws_elems,
               b->nslots);
    b->ws_bytes = (size_t)ws_elems * elem_bytes(b->dtype);
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
    if (b->d_ctl) { (void)hipFree(b->d_ctl); b->d_ctl = nullptr; }
    if (b->ws) { (void)hipFree(b->ws); b->ws = nullptr; }
    const size_t ib = std::max<size_t>(1, b->items.size()) * sizeof(HostBatchItem);
    const size_t ob = std::max<size_t>(1, b->offs.size()) * sizeof(int64_t);
    b->ctl_words = 2 + b->nslots;
    if ((e = hipMalloc(&b->d_items, ib)) != hipSuccess) return hip_error(e, "hipMalloc(items)");
    if ((e = hipMalloc(&b->d_offs, ob)) != hipSuccess) return hip_error(e, "hipMalloc(offsets)");
    if ((e = hipMalloc(&b->d_ctl, sizeof(unsigned) * b->ctl_words)) != hipSuccess)
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
    if ((e = hipMemset(b->d_ctl, 0, sizeof(unsigned) * b->ctl_words)) != hipSuccess)
        return hip_error(e, "hipMemset(control)");
    int resident = 0;
    if (batch_resident_grid(b->dtype, b->device, &resident) != FFT_OK) return FFT_EHIP;
    b->grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)b->items.size(), resident));
    return FFT_OK;
}

static void drop_graph(fft_batch* b) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    b->knode = nullptr;
    b->cap_in = nullptr;
    b->cap_out = nullptr;
}

// Captures reset + persistent kernel once on the plan's own stream.
static int capture(fft_batch* b, const void* in, void* out) {
    hipError_t e;
    if (!b->cap_stream && (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_error(e, "hipStreamCreate");
    if ((e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_error(e, "hipStreamBeginCapture");
    hipError_t le = launch_batch_reset(b->d_ctl, b->ctl_words, b->cap_stream);
    hipError_t lk = hipSuccess;
    if (le == hipSuccess)
        lk = launch_batch(b->dtype, in, out, b->ws, b->table->ptr, b->d_items, b->d_offs,
                          (int)b->items.size(), b->d_ctl, kSpinLimit, b->grid, b->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap_stream, &g);
    if (le != hipSuccess) return hip_error(le, "capture(reset)");
    if (lk != hipSuccess) return hip_error(lk, "capture(batch kernel)");
    if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
    b->graph = g;
    size_t nn = 0;
    if ((e = hipGraphGetNodes(g, nullptr, &nn)) != hipSuccess) return hip_error(e, "hipGraphGetNodes");
    std::vector<hipGraphNode_t> nodes(nn);
    if ((e = hipGraphGetNodes(g, nodes.data(), &nn)) != hipSuccess) return hip_error(e, "hipGraphGetNodes");
    for (auto nd : nodes) {
        hipGraphNodeType ty;
        if (hipGraphNodeGetType(nd, &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp;
        if (hipGraphKernelNodeGetParams(nd, &kp) != hipSuccess) continue;
        if (kp.func == batch_kernel_func(b->dtype)) b->knode = nd;
    }
    if (!b->knode) return set_error(FFT_EHIP, "batch kernel node not found in the captured graph");
    if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess)
        return hip_error(e, "hipGraphInstantiate");
    b->cap_in = in;
    b->cap_out = out;
    return FFT_OK;
}

// Points the captured kernel node at new data buffers.
static int retarget(fft_batch* b, const void* in, void* out) {
    hipKernelNodeParams kp;
    hipError_t e = hipGraphKernelNodeGetParams(b->knode, &kp);
    if (e != hipSuccess) return hip_error(e, "hipGraphKernelNodeGetParams");
    const void* a_in = in;
    void* a_out = out;
    void* a_ws = b->ws;
    const void* a_lt = b->table->ptr;
    const void* a_items = b->d_items;
    const int64_t* a_offs = b->d_offs;
    int a_n = (int)b->items.size();
    unsigned* a_ctl = b->d_ctl;
    int a_spin = kSpinLimit;
    void* args[] = {&a_in, &a_out, &a_ws, &a_lt, &a_items, &a_offs, &a_n, &a_ctl, &a_spin};
    kp.kernelParams = args;
    kp.extra = nullptr;
    if ((e = hipGraphExecKernelNodeSetParams(b->exec, b->knode, &kp)) != hipSuccess)
        return hip_error(e, "hipGraphExecKernelNodeSetParams");
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
    if (b->items.empty()) return FFT_OK;
    int rc = FFT_OK;
    if (!b->exec) rc = capture(b, in, out);
    else if (b->cap_in != in || b->cap_out != out) rc = retarget(b, in, out);
    if (rc != FFT_OK) return rc;
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
    if ((e = hipEventRecord(b->last, s)) != hipSuccess) return hip_error(e, "hipEventRecord");
    return FFT_OK;
}

fft_batch* batch_create(const int64_t* n, int64_t count, int dtype, int kind, const int* choice) {
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
    for (int m = 1; m <= 13; ++m) b->cfg_choice[m] = kSmallCfg[m];
    if (choice) {
        if (choice[0] == HB_N1024 || choice[0] == HB_N1024_B) b->cfg_choice[10] = choice[0];
        if (choice[1] == HB_N4096 || choice[1] == HB_N4096_B) b->cfg_choice[12] = choice[1];
    }
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        hip_error(e, "hipGetDevice");
        return nullptr;
    }
    if (get_table(nmax, dtype, kind, &b->table) != FFT_OK) return nullptr;
    build_items(b.get());
    if (upload(b.get()) != FFT_OK) return nullptr;
    if ((e = hipEventCreateWithFlags(&b->last, hipEventDisableTiming)) != hipSuccess) {
        hip_error(e, "hipEventCreate");
        return nullptr;
    }
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
    const int c[2] = {choice_1024 == 1 ? HB_N1024_B : HB_N1024,
                      choice_4096 == 1 ? HB_N4096_B : HB_N4096};
    return batch_create(n, count, (int)dtype, (int)kind, c);
}

int fft_batch_execute(fft_batch* b, const void* in, void* out, void* stream) {
    return batch_execute(b, in, out, (hipStream_t)stream);
}

int fft_batch_elements(const fft_batch* b, int64_t* elements) {
    if (!b || !elements) return set_error(FFT_EINVAL, "null argument");
    *elements = b->total;
    return FFT_OK;
}

int fft_batch_status(fft_batch* b, int* flags) {
    if (!b || !flags) return set_error(FFT_EINVAL, "null argument");
    hipError_t e = hipEventSynchronize(b->last);
    if (e != hipSuccess) return hip_error(e, "hipEventSynchronize");
    unsigned f = 0;
    if ((e = hipMemcpy(&f, b->d_ctl + 1, sizeof(unsigned), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_error(e, "hipMemcpy(status)");
    *flags = (int)f;
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

}  // extern "C"
