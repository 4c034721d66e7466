// C ABI of the dual-select FFT library (declared in include/dsfft.h): plans,
// table cache, schedule choice and launches.
#include "dsfft.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "fft_device.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "tables.hpp"

namespace dsfft {

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_error(hipError_t e, const char* where) {
    return set_error(FFT_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------- table cache

DeviceTable::~DeviceTable() {
    if (ptr) (void)hipFree(ptr);
}

static std::mutex g_table_mu;
static std::map<std::tuple<int, int, int, int>, std::shared_ptr<DeviceTable>> g_tables;

// Level-ordered table with capacity >= n for (device, dtype, kind), shared by
// every plan that needs it.  A larger request replaces the cached table; plans
// holding the old one keep it alive.
static std::vector<std::shared_ptr<DeviceTable>> g_retired_tables;

int get_table(int64_t n, int dtype, int kind, bool inverse, std::shared_ptr<DeviceTable>* out, int radix) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_table_mu);
    auto key = std::make_tuple(dev, dtype, kind, (int)inverse | (radix == 4 ? 2 : 0));
    auto it = g_tables.find(key);
    if (it != g_tables.end() && it->second->ncap >= n) {
        *out = it->second;
        return FFT_OK;
    }
    const int64_t ncap = std::max<int64_t>(n, kMinTableEntries);
    std::vector<uint8_t> img = radix == 4 ? build_level_table4(ncap, dtype, kind, inverse)
                                          : build_level_table(ncap, dtype, kind, inverse);
    auto t = std::make_shared<DeviceTable>();
    t->ncap = ncap;
    t->bytes = img.size();
    e = hipMalloc(&t->ptr, img.size());
    if (e != hipSuccess) {
        t->ptr = nullptr;
        return e == hipErrorOutOfMemory ? set_error(FFT_ENOMEM, "table allocation failed")
                                        : hip_error(e, "hipMalloc(table)");
    }
    e = hipMemcpy(t->ptr, img.data(), img.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "hipMemcpy(table)");
    // A replaced (smaller) table is kept until the process ends: kernels
    // already enqueued by plans of any lifetime may still read it, and plans
    // do not wait for their last launch when they are destroyed.  Capacities
    // grow by powers of two, so all retired tables together are smaller than
    // the current one.
    if (it != g_tables.end()) g_retired_tables.push_back(it->second);
    g_tables[key] = t;
    *out = t;
    return FFT_OK;
}

// ------------------------------------------------------------ kernel choice

static const KernelCfg* table_for(int dtype, int* count) {
    return dtype == DT_F16 ? kernel_table_f16(count)
                           : (dtype == DT_F32 ? kernel_table_f32(count) : kernel_table_f16f32(count));
}

const KernelCfg* find_kernel(int dtype, int mode, int log_nu, int variant, bool radix4) {
    int cnt = 0;
    const KernelCfg* t = table_for(dtype, &cnt);
    int seen = 0;
    for (int i = 0; i < cnt; ++i) {
        if (t[i].mode != mode || t[i].log_nu != log_nu) continue;
        if ((t[i].encoding == ENC_RADIX4) != radix4) continue;
        if (t[i].lds_bytes > 160 * 1024) continue;
        if (seen++ == variant) return &t[i];
    }
    return nullptr;
}

// First configuration of (dtype, mode, log_nu) that does not stage through
// LDS with 16-byte accesses (used when data pointers are not 16-byte aligned).
const KernelCfg* find_plain_kernel(int dtype, int mode, int log_nu, bool radix4 = false) {
    for (int v = 0;; ++v) {
        const KernelCfg* k = find_kernel(dtype, mode, log_nu, v, radix4);
        if (!k || !k->staged) return k;
    }
}

int count_kernels(int dtype, int mode, int log_nu, bool radix4) {
    int n = 0;
    while (find_kernel(dtype, mode, log_nu, n, radix4)) ++n;
    return n;
}

std::string describe(const KernelCfg* k) {
    if (!k) return "none";
    static const char* modes[] = {"small", "cols", "rows"};
    char buf[160];
    std::snprintf(buf, sizeof buf,
                  "%s:nu=2^%d,e=2^%d,upw=%d,r=[%d,%d,%d],stg=%d,lane=%d,pipe=%d,t=%d,lds=%zu",
                  modes[k->mode], k->log_nu, k->log_e, k->upw, k->lr[0], k->lr[1], k->lr[2],
                  k->staged, k->lane_tail, k->pipelined, k->threads, k->lds_bytes);
    std::string d = buf;
    if (k->upl > 1) d += ",upl=" + std::to_string(k->upl);
    if (k->encoding == ENC_RADIX4) d += ",radix4";
    else if (k->encoding) d += k->encoding == ENC_SELECT ? ",enc=select" : ",enc=branch";
    return d;
}

// Largest single-kernel size per dtype: the largest whole-transform
// configuration that fits (binary16 2^16 points, whose exchanges run in two
// rounds through LDS; binary32 and binary16 storage with binary32 butterflies
// 2^15); beyond it, the two-pass split.  A tuning record may still choose the
// split for a size that has a whole-transform configuration.
static int small_limit(int dtype) {
    int m = 20;
    while (m > 0 && count_kernels(dtype, MODE_SMALL, m) == 0) --m;
    return m;
}

// Small batches: the default and tuned configurations hold several
// transforms per workgroup (tuned on 256 MiB batches).  When a launch would
// have fewer workgroups than the device has compute units, its time is one
// workgroup's walk through its transforms; the first plain configuration with
// one transform per workgroup, where the size has one, finishes sooner
// (binary32 N = 1024 x 16: 4.4 against 5.6 us per kernel; binary16 3.3 us).
static void small_batch_choice(fft_plan* p) {
    if (p->k2 || !p->k1 || p->k1->upw == 1) return;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) return;
    if ((p->batch + p->k1->upw - 1) / p->k1->upw >= cus) return;
    for (int v = 0;; ++v) {
        const KernelCfg* k = find_kernel(p->dtype, MODE_SMALL, p->log_n, v);
        if (!k) return;
        if (k->upw == 1 && !k->staged && !k->lane_tail && !k->pipelined && !k->encoding) {
            p->k1 = k;
            p->k1_plain = k;
            return;
        }
    }
}

int choose_schedule(fft_plan* p, const int* variants) {
    const int m = p->log_n;
    const int v0 = variants ? variants[0] : 0, v1 = variants ? variants[1] : 0;
    if (p->radix == 4) {
        // the radix-4 form runs whole transforms only
        p->k1 = find_kernel(p->dtype, MODE_SMALL, m, v0, true);
        p->k1_plain = find_plain_kernel(p->dtype, MODE_SMALL, m, true);
        p->k2 = nullptr;
        if (!p->k1 || !p->k1_plain) return set_error(FFT_EUNSUPPORTED, "no radix-4 kernel for this size and dtype");
        return FFT_OK;
    }
    if (m <= small_limit(p->dtype) && (!variants || variants[2] == 0)) {
        p->k1 = find_kernel(p->dtype, MODE_SMALL, m, v0);
        p->k1_plain = find_plain_kernel(p->dtype, MODE_SMALL, m);
        p->k2 = nullptr;
        if (!p->k1 || !p->k1_plain) return set_error(FFT_EUNSUPPORTED, "no kernel for this size");
        return FFT_OK;
    }
    const int m1 = (m + 1) / 2, m2 = m - m1;     // columns of 2^m1, rows of 2^m2
    p->k1 = find_kernel(p->dtype, MODE_COLS, m1, v0);
    p->k1_plain = p->k1;
    p->k2 = find_kernel(p->dtype, MODE_ROWS, m2, v1);
    if (!p->k1 || !p->k2) return set_error(FFT_EUNSUPPORTED, "no two-pass kernels for this size");
    return FFT_OK;
}

// Bytes of a stored element (the plan's input and output) and of a two-pass
// intermediate element (the compute precision).
int elem_bytes(int dtype) { return dtype == DT_F32 ? 8 : 4; }
int work_elem_bytes(int dtype) { return dtype == DT_F16 ? 4 : 8; }

// Workspace: two-pass schedules stage the intermediate per chunk of
// transforms, capped at 128 MiB (measured: 128 MiB chunks run 5-6 % faster
// than 64 MiB or 1 GiB ones; 8 MiB chunks take twice as long, the kernels
// being too short for their launch and tail).
void size_workspace(fft_plan* p) {
    if (!p->k2) {
        p->chunk = p->batch;
        p->ws_need = 0;
        return;
    }
    const size_t per = (size_t)p->n * work_elem_bytes(p->dtype);
    const size_t cap = kMaxWorkspaceBytes;
    int64_t chunk = (int64_t)std::max<size_t>(1, cap / per);
    chunk = std::min<int64_t>(chunk, p->batch);
    p->chunk = chunk;
    p->ws_need = (size_t)chunk * per;
}

// The plan's launches with the two-pass intermediate in `ws`, `chunk`
// transforms at a time (fft_execute: the plan's workspace and chunk).
int launch_plan_ws(const fft_plan* p, const void* in, void* out, hipStream_t s, void* ws, int64_t chunk) {
    const void* lt = p->table->ptr;
    if (!p->k2) {
        const bool aligned16 = (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
        const KernelCfg* k = (p->k1->staged && !aligned16) ? p->k1_plain : p->k1;
        hipError_t e = k->launch(in, out, lt, p->batch, 0, s);
        if (e != hipSuccess) return hip_error(e, "launch");
        return FFT_OK;
    }
    const int m1 = p->k1->log_nu, m2 = p->k2->log_nu;
    const size_t eb = (size_t)elem_bytes(p->dtype);
    for (int64_t b0 = 0; b0 < p->batch; b0 += chunk) {
        const int64_t nb = std::min<int64_t>(chunk, p->batch - b0);
        const char* src = (const char*)in + (size_t)b0 * p->n * eb;
        char* dst = (char*)out + (size_t)b0 * p->n * eb;
        hipError_t e = p->k1->launch(src, ws, lt, nb << m2, m2, s);
        if (e != hipSuccess) return hip_error(e, "launch(cols)");
        e = p->k2->launch(ws, dst, lt, nb << m1, m1, s);
        if (e != hipSuccess) return hip_error(e, "launch(rows)");
    }
    return FFT_OK;
}

int launch_plan(fft_plan* p, const void* in, void* out, hipStream_t s) {
    return launch_plan_ws(p, in, out, s, p->ws, p->chunk);
}

static bool is_pow2(int64_t n) { return n >= 2 && (n & (n - 1)) == 0; }

fft_plan* plan_create(int64_t n, int64_t batch, int dtype, int kind, const int* variants,
                      bool inverse, int radix, bool alloc_ws) {
    if (!is_pow2(n) || n > (int64_t(1) << 20)) {
        set_error(FFT_EINVAL, "n must be a power of two in [2, 2^20]");
        return nullptr;
    }
    if (batch < 1) {
        set_error(FFT_EINVAL, "batch must be >= 1");
        return nullptr;
    }
    if (dtype != DT_F16 && dtype != DT_F32 && dtype != DT_F16F32) {
        set_error(FFT_EINVAL, "dtype must be FFT_F16, FFT_F32 or FFT_F16_F32");
        return nullptr;
    }
    if (kind < 0 || kind > 3) {
        set_error(FFT_EINVAL, "unknown table kind");
        return nullptr;
    }
    std::unique_ptr<fft_plan> p(new fft_plan());
    p->n = n;
    p->batch = batch;
    p->dtype = dtype;
    p->kind = kind;
    p->inverse = inverse;
    p->radix = radix;
    p->log_n = 0;
    while ((int64_t(1) << p->log_n) < n) ++p->log_n;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        hip_error(e, "hipGetDevice");
        return nullptr;
    }
    if (get_table(n, table_dtype(dtype), kind, inverse, &p->table, radix) != FFT_OK) return nullptr;
    int tuned[3];
    if (!variants && radix == 2 && tuned_choice(dtype, p->log_n, tuned)) {
        // a recorded tuning choice; fall back to the fixed rule if it no longer exists
        if (choose_schedule(p.get(), tuned) != FFT_OK && choose_schedule(p.get(), nullptr) != FFT_OK)
            return nullptr;
    } else if (choose_schedule(p.get(), variants) != FFT_OK) {
        return nullptr;
    }
    if (!variants && radix == 2) small_batch_choice(p.get());
    size_workspace(p.get());
    if (p->ws_need && alloc_ws) {
        e = hipMalloc(&p->ws, p->ws_need);
        if (e != hipSuccess) {
            p->ws = nullptr;
            set_error(e == hipErrorOutOfMemory ? FFT_ENOMEM : FFT_EHIP, "workspace allocation failed");
            return nullptr;
        }
        p->ws_owned = true;
        p->ws_bytes = p->ws_need;
    }
    return p.release();
}

static bool ranges_partially_overlap(const void* a, const void* b, size_t bytes) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    if (x == y) return false;
    return x < y + bytes && y < x + bytes;
}

int check_execute_args(const fft_plan* p, const void* in, const void* out) {
    if (!p) return set_error(FFT_EINVAL, "null plan");
    if (!in || !out) return set_error(FFT_EINVAL, "null data pointer");
    const size_t eb = (size_t)elem_bytes(p->dtype);
    if (((uintptr_t)in % eb) || ((uintptr_t)out % eb))
        return set_error(FFT_EINVAL, "data pointers must be aligned to the element size");
    if (ranges_partially_overlap(in, out, (size_t)p->n * p->batch * eb))
        return set_error(FFT_EINVAL, "in and out partially overlap");
    return FFT_OK;
}

int plan_execute(fft_plan* p, const void* in, void* out, hipStream_t s) {
    int rc = check_execute_args(p, in, out);
    if (rc != FFT_OK) return rc;
    return launch_plan(p, in, out, s);
}

// Frees a plan-owned workspace once the plan's device has finished all work
// enqueued so far (any launch of the plan may still read or write it).  An
// event recorded per execute would say exactly when its last launch ends, but
// costs several microseconds of device time per execute (≈ 12 us per
// two-pass execute measured); freeing happens once per plan.
void release_workspace(fft_plan* p) {
    if (!p->ws || !p->ws_owned) return;
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    if (have_cur && cur != p->device) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(p->ws);
    if (have_cur && cur != p->device) (void)hipSetDevice(cur);
    p->ws = nullptr;
    p->ws_owned = false;
}

}  // namespace dsfft

fft_plan::~fft_plan() { dsfft::release_workspace(this); }

using namespace dsfft;

extern "C" {

const char* fft_last_error(void) { return g_last_error.c_str(); }

fft_plan* fft_plan_create(int64_t n, int64_t batch, fft_dtype dtype, fft_table_kind kind) {
    return plan_create(n, batch, (int)dtype, (int)kind, nullptr);
}

fft_plan* fft_plan_create_dir(int64_t n, int64_t batch, fft_dtype dtype, fft_table_kind kind,
                              int direction) {
    if (direction != FFT_FORWARD && direction != FFT_INVERSE) {
        set_error(FFT_EINVAL, "direction must be FFT_FORWARD or FFT_INVERSE");
        return nullptr;
    }
    return plan_create(n, batch, (int)dtype, (int)kind, nullptr, direction == FFT_INVERSE);
}

int fft_execute(fft_plan* plan, const void* in, void* out, void* stream) {
    return plan_execute(plan, in, out, (hipStream_t)stream);
}

void fft_destroy(fft_plan* plan) { delete plan; }

int fft_table_build_dir(int64_t n, fft_dtype dtype, fft_table_kind kind, int direction,
                        void* mult_out, void* ratio_out, uint8_t* path_out) {
    if (n < 2 || (n & (n - 1)) || n > (int64_t(1) << 20))
        return set_error(FFT_EINVAL, "n must be a power of two in [2, 2^20]");
    if ((int)dtype != DT_F16 && (int)dtype != DT_F32) return set_error(FFT_EINVAL, "bad dtype");
    if ((int)kind < 0 || (int)kind > 3) return set_error(FFT_EINVAL, "bad table kind");
    if (direction != FFT_FORWARD && direction != FFT_INVERSE)
        return set_error(FFT_EINVAL, "direction must be FFT_FORWARD or FFT_INVERSE");
    build_flat_table(n, (int)dtype, (int)kind, direction == FFT_INVERSE, mult_out, ratio_out,
                     path_out);
    return FFT_OK;
}

int fft_table_build(int64_t n, fft_dtype dtype, fft_table_kind kind, void* mult_out,
                    void* ratio_out, uint8_t* path_out) {
    return fft_table_build_dir(n, dtype, kind, FFT_FORWARD, mult_out, ratio_out, path_out);
}

int fft_plan_info(const fft_plan* p, int64_t* n, int64_t* batch, int* dtype, int* kind,
                  char* config_out, size_t cap) {
    if (!p) return set_error(FFT_EINVAL, "null plan");
    if (n) *n = p->n;
    if (batch) *batch = p->batch;
    if (dtype) *dtype = p->dtype;
    if (kind) *kind = p->kind;
    if (config_out && cap) {
        std::string d = describe(p->k1);
        if (p->k2) d += " | " + describe(p->k2) + " | chunk=" + std::to_string(p->chunk);
        std::snprintf(config_out, cap, "%s", d.c_str());
    }
    return FFT_OK;
}

int fft_plan_workspace_bytes(const fft_plan* p, size_t* bytes) {
    if (!p || !bytes) return set_error(FFT_EINVAL, "null argument");
    *bytes = p->ws_need;
    return FFT_OK;
}

int fft_plan_set_workspace(fft_plan* p, void* dev_ptr, size_t bytes) {
    if (!p) return set_error(FFT_EINVAL, "null plan");
    if (p->ws_need == 0) return FFT_OK;
    if (!dev_ptr || bytes < p->ws_need || ((uintptr_t)dev_ptr % 16))
        return set_error(FFT_EINVAL, "workspace too small, null or misaligned");
    release_workspace(p);
    p->ws = dev_ptr;
    p->ws_bytes = bytes;
    p->ws_owned = false;
    return FFT_OK;
}

}  // extern "C"

extern "C" {

fft_plan* fft_plan_create_radix4(int64_t n, int64_t batch, fft_dtype dtype, fft_table_kind kind,
                                 int direction, int variant) {
    if (direction != FFT_FORWARD && direction != FFT_INVERSE) {
        set_error(FFT_EINVAL, "direction must be FFT_FORWARD or FFT_INVERSE");
        return nullptr;
    }
    if ((int)dtype == DT_F16F32) {
        set_error(FFT_EUNSUPPORTED, "the radix-4 form takes FFT_F16 or FFT_F32");
        return nullptr;
    }
    if (variant < -1) {
        set_error(FFT_EINVAL, "variant must be -1 (default) or a configuration index");
        return nullptr;
    }
    const int v[3] = {variant < 0 ? 0 : variant, 0, 0};
    return plan_create(n, batch, (int)dtype, (int)kind, v, direction == FFT_INVERSE, 4);
}

int fft_config_count_radix4(int64_t n, fft_dtype dtype, int* count) {
    if (n < 2 || (n & (n - 1)) || n > (int64_t(1) << 20))
        return set_error(FFT_EINVAL, "n must be a power of two in [2, 2^20]");
    if (!count) return set_error(FFT_EINVAL, "null argument");
    if ((int)dtype != DT_F16 && (int)dtype != DT_F32 && (int)dtype != DT_F16F32)
        return set_error(FFT_EINVAL, "bad dtype");
    int m = 0;
    while ((int64_t(1) << m) < n) ++m;
    *count = (int)dtype == DT_F16F32 ? 0 : count_kernels((int)dtype, MODE_SMALL, m, true);
    return FFT_OK;
}

int fft_table_build_radix4(int64_t n, fft_dtype dtype, fft_table_kind kind, int direction,
                           void* mult_out, void* ratio_out, uint8_t* path_out, void* rho_out,
                           uint8_t* sel_out) {
    if (n < 4 || (n & (n - 1)) || n > (int64_t(1) << 20))
        return set_error(FFT_EINVAL, "n must be a power of two in [4, 2^20]");
    if ((int)dtype != DT_F16 && (int)dtype != DT_F32) return set_error(FFT_EINVAL, "bad dtype");
    if ((int)kind < 0 || (int)kind > 3) return set_error(FFT_EINVAL, "bad table kind");
    if (direction != FFT_FORWARD && direction != FFT_INVERSE)
        return set_error(FFT_EINVAL, "direction must be FFT_FORWARD or FFT_INVERSE");
    build_flat_table4(n, (int)dtype, (int)kind, direction == FFT_INVERSE, mult_out, ratio_out, path_out,
                      rho_out, sel_out);
    return FFT_OK;
}

fft_plan* fft_plan_create_variant(int64_t n, int64_t batch, fft_dtype dtype, fft_table_kind kind,
                                  int variant_a, int variant_b, int two_pass) {
    if (variant_a < 0 || variant_b < 0) {
        set_error(FFT_EINVAL, "negative variant");
        return nullptr;
    }
    const int v[3] = {variant_a, variant_b, two_pass ? 1 : 0};
    return plan_create(n, batch, (int)dtype, (int)kind, v);
}

int fft_config_count(int64_t n, fft_dtype dtype, int* single, int* cols, int* rows) {
    if (n < 2 || (n & (n - 1)) || n > (int64_t(1) << 20))
        return set_error(FFT_EINVAL, "n must be a power of two in [2, 2^20]");
    if ((int)dtype != DT_F16 && (int)dtype != DT_F32 && (int)dtype != DT_F16F32)
        return set_error(FFT_EINVAL, "bad dtype");
    int m = 0;
    while ((int64_t(1) << m) < n) ++m;
    const int m1 = (m + 1) / 2, m2 = m - m1;
    if (single) *single = count_kernels((int)dtype, MODE_SMALL, m);
    if (cols) *cols = count_kernels((int)dtype, MODE_COLS, m1);
    if (rows) *rows = count_kernels((int)dtype, MODE_ROWS, m2);
    return FFT_OK;
}

}  // extern "C"
