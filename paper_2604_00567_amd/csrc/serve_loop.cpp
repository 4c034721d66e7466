// Native serving loops over an arrival trace, and the request payload
// generator they share.
//
//   continuous     K slots on K streams; requests are admitted in arrival order
//                  into a free slot while they fit the HBM budget and the
//                  slot's capacities, and each slot runs one step per
//                  precision (the serving-slot batch kernels, or, for a step of
//                  at most direct_max requests, one cached-plan launch per
//                  request); steps on different slots overlap.
//   per request    one cached-plan launch per request, round-robin over K
//                  streams, admitted in arrival order under the same budget.
//
// Latency of a request = the host time at which its completion is observed
// minus its scheduled arrival time.  Payloads are generated on the device:
// request r of precision d holds N(0, 1) values keyed by (seed, d, its
// position in the concatenation of that precision's requests in arrival
// order), so a request's data do not depend on how requests are grouped.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "batch_launch.hpp"
#include "dsfft.h"
#include "plan.hpp"
#include "tables.hpp"

namespace dsfft {
namespace {

// ----------------------------------------------------------- payload generator

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): ten rounds of two 32 x 32 -> 64-bit products on
// the counter, key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Element `first + e` of precision stream `dt`: (re, im) = one Box-Muller pair
// of the counter (first + e, dt); uniforms in (0, 1) from the top 24 bits.
template <class T>
__global__ void fill_normal_kernel(T* out, int64_t elems, uint64_t first, uint32_t dt, uint64_t seed) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < elems; e += step) {
        const uint64_t idx = first + (uint64_t)e;
        uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), dt, 0x5EEDu};
        philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const float u1 = ((float)(c[0] >> 8) + 0.5f) * (1.0f / 16777216.0f);
        const float u2 = ((float)(c[1] >> 8) + 0.5f) * (1.0f / 16777216.0f);
        const float r = sqrtf(-2.0f * logf(u1));
        float s, co;
        sincosf(6.283185307179586f * u2, &s, &co);
        out[2 * e] = (T)(r * co);
        out[2 * e + 1] = (T)(r * s);
    }
}

hipError_t fill_normal(int dtype, void* data, int64_t elems, uint64_t first, uint64_t seed, hipStream_t st) {
    if (elems <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((elems + 255) / 256, 4096);
    if (dtype == DT_F16)
        hipLaunchKernelGGL(fill_normal_kernel<_Float16>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (_Float16*)data, elems, first, 0u, seed);
    else
        hipLaunchKernelGGL(fill_normal_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, (float*)data,
                           elems, first, 1u, seed);
    return hipGetLastError();
}

// ------------------------------------------------------------------ helpers

using Clock = std::chrono::steady_clock;

inline int dt_index(int dtype) { return dtype == DT_F16 ? 0 : 1; }
inline size_t ebytes(int dtype) { return dtype == DT_F16 ? 4 : 8; }
inline bool is_split(int64_t n, int dtype) { return n > (int64_t(1) << max_whole_log(dtype)); }

// What a step holds so far, per precision: elements, whole transforms, split
// transforms and their elements, transforms per size and the work items they
// make (the slot's capacity checks).
struct StepLoad {
    int64_t used[2] = {0, 0}, whole[2] = {0, 0}, large[2] = {0, 0}, large_elems[2] = {0, 0};
    int64_t per_size[2][19] = {}, items[2] = {0, 0};
};

inline int log2_of(int64_t n) {
    int m = 0;
    while ((int64_t(1) << m) < n) ++m;
    return m;
}

struct Trace {
    const double* t;
    const int64_t* n;
    const int64_t* b;
    const int32_t* dtype;
    int64_t count;
};

// Plans per (shape, key).  With a workspace for the key (one per stream in
// the per-request loop), two-pass plans share it instead of owning their own:
// launches on one stream are ordered, so they never use it at the same time.
// The continuous loop keys every plan 0 and launches a two-pass plan on the
// workspace of the slot that runs it.
struct PlanCache {
    std::map<std::tuple<int64_t, int64_t, int, int>, fft_plan*> plans;
    int kind = 0;
    std::vector<void*> ws;      // per key (may be empty)
    fft_plan* get(int64_t n, int64_t b, int dtype, int key) {
        auto k = std::make_tuple(n, b, dtype, key);
        auto it = plans.find(k);
        if (it != plans.end()) return it->second;
        const bool shared = key < (int)ws.size() && ws[key];
        fft_plan* p = plan_create(n, b, dtype, kind, nullptr, false, 2, !shared);
        if (!p) return nullptr;
        if (shared && p->ws_need) {
            p->ws = ws[key];
            p->ws_bytes = kMaxWorkspaceBytes;
            p->ws_owned = false;
        }
        plans[k] = p;
        return p;
    }
    ~PlanCache() {
        for (auto& kv : plans) delete kv.second;
    }
};

struct EventPool {
    std::vector<hipEvent_t> free;
    std::vector<hipEvent_t> all;
    hipError_t get(hipEvent_t* e) {
        if (!free.empty()) {
            *e = free.back();
            free.pop_back();
            return hipSuccess;
        }
        hipError_t r = hipEventCreateWithFlags(e, hipEventDisableTiming);
        if (r == hipSuccess) all.push_back(*e);
        return r;
    }
    void put(hipEvent_t e) { free.push_back(e); }
    ~EventPool() {
        for (hipEvent_t e : all) (void)hipEventDestroy(e);
    }
};

}  // namespace

// Admission of one step (continuous loop): requests from `head` on, in arrival
// order, while each fits the budget (request bytes, plus workspace for split
// transforms, on top of what is in flight) and the step's capacities.
// At most `limit` requests (and max_step_requests).
int64_t serve_admit(const Trace& tr, const int64_t* order, int64_t avail, int64_t head, size_t inflight,
                    const fft_serve_config& c, std::vector<int64_t>& take, size_t* inflight_out,
                    int64_t limit) {
    StepLoad ld;
    take.clear();
    limit = std::min<int64_t>(limit, c.max_step_requests);
    while (head < avail && (int64_t)take.size() < limit) {
        const int64_t r = order[head];
        const int64_t n = tr.n[r], b = tr.b[r];
        const int dt = tr.dtype[r], d = dt_index(dt);
        const size_t eb = ebytes(dt);
        const size_t nb = 2 * (size_t)n * b * eb;
        const size_t ws = is_split(n, dt) ? (size_t)n * b * eb : 0;
        if (inflight + nb + ws > c.budget_bytes) break;
        const int64_t elems = n * b;
        const int64_t cap = (int64_t)(c.slot_bytes / eb);
        if (ld.used[d] + elems > cap) break;
        // work items of the slot's kernels (split transforms take none when
        // they run through their plans)
        const int m = log2_of(n);
        const int64_t cnt = ld.per_size[d][m];
        const int64_t more = c.split_direct && is_split(n, dt)
                                 ? 0
                                 : work_items_of_class(dt, m, cnt + b) - work_items_of_class(dt, m, cnt);
        if (ld.items[d] + more > c.max_items) break;
        if (is_split(n, dt)) {
            if (ld.large[d] + b > c.max_large || (size_t)(ld.large_elems[d] + elems) * eb > c.slot_bytes) break;
            ld.large[d] += b;
            ld.large_elems[d] += elems;
        } else {
            if (ld.whole[d] + b > c.max_transforms) break;
            ld.whole[d] += b;
        }
        ld.per_size[d][m] += b;
        ld.items[d] += more;
        ld.used[d] += elems;
        take.push_back(r);
        inflight += nb;
        ++head;
    }
    *inflight_out = inflight;
    return head;
}

}  // namespace dsfft

using namespace dsfft;

namespace {

struct Slot {
    hipStream_t st = nullptr;
    void* arena[2] = {nullptr, nullptr};
    fft_serve_slot* native[2] = {nullptr, nullptr};
    hipEvent_t done = nullptr;
    hipEvent_t early = nullptr;      // the step's whole-size requests (split_direct)
    bool busy = false, early_busy = false;
    std::vector<int64_t> rids, early_rids;
};

// One precision's requests of a step, in admission order, with their element
// offsets in the slot's arena.
struct Group {
    std::vector<int64_t> rid, n, b, off;
    void clear() {
        rid.clear();
        n.clear();
        b.clear();
        off.clear();
    }
    void add(int64_t r, int64_t nn, int64_t bb, int64_t o) {
        rid.push_back(r);
        n.push_back(nn);
        b.push_back(bb);
        off.push_back(o);
    }
};

struct Inflight {
    int64_t rid;
    hipEvent_t ev;
    int stream;
    size_t off, len;      // ring span
};

// Ring of device memory per stream: requests on one stream complete in order,
// so spans are freed first in, first out.
struct Ring {
    char* base = nullptr;
    size_t cap = 0, head = 0, used = 0;
    std::deque<std::pair<size_t, size_t>> spans;   // (offset, length incl. skipped tail)
    bool alloc(size_t len, size_t* off) {
        len = (len + 255) & ~size_t(255);
        if (len > cap) return false;
        size_t start = head, skip = 0;
        if (start + len > cap) {        // wrap: skip the tail
            skip = cap - start;
            start = 0;
        }
        if (used + skip + len > cap) return false;
        *off = start;
        spans.emplace_back(start, skip + len);
        used += skip + len;
        head = start + len;
        if (head == cap) head = 0;
        return true;
    }
    void release_front() {
        used -= spans.front().second;
        spans.pop_front();
        if (spans.empty()) head = used = 0;
    }
};

double seconds_since(Clock::time_point t0) {
    return std::chrono::duration<double>(Clock::now() - t0).count();
}

}  // namespace

extern "C" {

int fft_serve_fill(fft_dtype dtype, void* data, int64_t elems, uint64_t first, uint64_t seed, void* stream) {
    if ((int)dtype != DT_F16 && (int)dtype != DT_F32) return set_error(FFT_EINVAL, "dtype must be FFT_F16 or FFT_F32");
    if (!data || elems < 0) return set_error(FFT_EINVAL, "null data or negative size");
    hipError_t e = fill_normal((int)dtype, data, elems, first, seed, (hipStream_t)stream);
    return e == hipSuccess ? FFT_OK : hip_error(e, "launch(fill)");
}

int fft_serve_admit(const int64_t* n, const int64_t* batch, const int32_t* dtype, int64_t count,
                    int64_t head, size_t inflight_bytes, const fft_serve_config* cfg, int64_t* taken,
                    int64_t* ntaken, size_t* inflight_out) {
    if (!n || !batch || !dtype || !cfg || !taken || !ntaken || !inflight_out || head < 0 || count < 0)
        return set_error(FFT_EINVAL, "null argument");
    for (int64_t r = 0; r < count; ++r) {
        if (n[r] < 2 || (n[r] & (n[r] - 1)) || n[r] > (int64_t(1) << 18) || batch[r] < 1)
            return set_error(FFT_EINVAL, "request sizes must be powers of two in [2, 2^18], batch >= 1");
        if (dtype[r] != DT_F16 && dtype[r] != DT_F32) return set_error(FFT_EINVAL, "request dtype must be FFT_F16 or FFT_F32");
    }
    std::vector<int64_t> order(count), take;
    for (int64_t i = 0; i < count; ++i) order[i] = i;
    Trace tr{nullptr, n, batch, dtype, count};
    serve_admit(tr, order.data(), count, head, inflight_bytes, *cfg, take, inflight_out, cfg->max_step_requests);
    std::copy(take.begin(), take.end(), taken);
    *ntaken = (int64_t)take.size();
    return FFT_OK;
}

int fft_serve_run(const fft_serve_config* cfg, const double* t, const int64_t* n, const int64_t* batch,
                  const int32_t* dtype, int64_t count, double* done_t, fft_serve_stats* stats,
                  void* out_dev, const int64_t* out_off) {
    if (!cfg || !t || !n || !batch || !dtype || !done_t || count < 0)
        return set_error(FFT_EINVAL, "null argument");
    const fft_serve_config c = *cfg;
    if (c.slots < 1 || c.slots > 64 || c.budget_bytes == 0 || c.max_step_requests < 1)
        return set_error(FFT_EINVAL, "bad serving configuration");
    if (c.mode != FFT_SERVE_CONTINUOUS && c.mode != FFT_SERVE_PER_REQUEST)
        return set_error(FFT_EINVAL, "mode must be FFT_SERVE_CONTINUOUS or FFT_SERVE_PER_REQUEST");
    if (c.mode == FFT_SERVE_CONTINUOUS && (c.slot_bytes == 0 || c.max_transforms < 1 || c.max_large < 0))
        return set_error(FFT_EINVAL, "bad slot capacities");
    Trace tr{t, n, batch, dtype, count};
    // sizes, precisions, arrival order and each request's generator offset
    std::vector<uint64_t> first(count);
    uint64_t vpos[2] = {0, 0};
    size_t max_req = 0;
    for (int64_t r = 0; r < count; ++r) {
        if (n[r] < 2 || (n[r] & (n[r] - 1)) || n[r] > (int64_t(1) << 18) || batch[r] < 1)
            return set_error(FFT_EINVAL, "request sizes must be powers of two in [2, 2^18], batch >= 1");
        if (dtype[r] != DT_F16 && dtype[r] != DT_F32) return set_error(FFT_EINVAL, "request dtype must be FFT_F16 or FFT_F32");
        if (r > 0 && t[r] < t[r - 1]) return set_error(FFT_EINVAL, "arrival times must not decrease");
        const int d = dt_index(dtype[r]);
        first[r] = vpos[d];
        vpos[d] += (uint64_t)(n[r] * batch[r]);
        max_req = std::max(max_req, (size_t)n[r] * batch[r] * ebytes(dtype[r]));
        done_t[r] = -1.0;
    }
    fft_serve_stats st{};
    hipError_t e;
    PlanCache plans;
    plans.kind = c.kind;
    EventPool events;
    std::vector<int64_t> order(count);
    for (int64_t i = 0; i < count; ++i) order[i] = i;

    if (c.mode == FFT_SERVE_CONTINUOUS) {
        std::vector<Slot> slots(c.slots);
        int rc = FFT_OK;
        auto cleanup = [&]() {
            for (auto& s : slots) {
                if (s.st) (void)hipStreamSynchronize(s.st);
                for (int d = 0; d < 2; ++d) {
                    if (s.native[d]) fft_serve_slot_destroy(s.native[d]);
                    if (s.arena[d]) (void)hipFree(s.arena[d]);
                }
                if (s.done) (void)hipEventDestroy(s.done);
                if (s.early) (void)hipEventDestroy(s.early);
                if (s.st) (void)hipStreamDestroy(s.st);
            }
            for (void* w : plans.ws) (void)hipFree(w);
            plans.ws.clear();
        };
        for (auto& s : slots) {
            if ((e = hipStreamCreate(&s.st)) != hipSuccess || (e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&s.early, hipEventDisableTiming)) != hipSuccess) {
                cleanup();
                return hip_error(e, "slot stream/event");
            }
            // workspace of the slot's direct two-pass launches (its steps are
            // ordered on its stream)
            void* w = nullptr;
            if ((e = hipMalloc(&w, kMaxWorkspaceBytes)) != hipSuccess) {
                cleanup();
                return set_error(e == hipErrorOutOfMemory ? FFT_ENOMEM : FFT_EHIP, "workspace allocation failed");
            }
            plans.ws.push_back(w);
            for (int d = 0; d < 2; ++d) {
                const int dt = d == 0 ? DT_F16 : DT_F32;
                if ((e = hipMalloc(&s.arena[d], c.slot_bytes)) != hipSuccess) {
                    cleanup();
                    return set_error(e == hipErrorOutOfMemory ? FFT_ENOMEM : FFT_EHIP, "slot arena allocation failed");
                }
                s.native[d] = fft_serve_slot_create((fft_dtype)dt, (fft_table_kind)c.kind, c.max_items,
                                                    c.max_transforms, c.max_large, c.slot_bytes);
                if (!s.native[d]) {
                    cleanup();
                    return FFT_ENOMEM;
                }
            }
        }
        if ((e = hipDeviceSynchronize()) != hipSuccess) {
            cleanup();
            return hip_error(e, "hipDeviceSynchronize");
        }
        int64_t nxt = 0, head = 0, completed = 0;
        size_t inflight = 0;
        size_t first_slot = 0;      // free slots are taken round-robin from here
        std::vector<int64_t> take;
        Group whole[2], split[2];
        double sum_req = 0;
        const Clock::time_point t0 = Clock::now();
        auto retire = [&](std::vector<int64_t>& rids) {
            const double td = seconds_since(t0);
            for (int64_t r : rids) {
                done_t[r] = td;
                inflight -= 2 * (size_t)n[r] * batch[r] * ebytes(dtype[r]);
            }
            completed += (int64_t)rids.size();
            rids.clear();
        };
        while (completed < count && rc == FFT_OK) {
            const double now = seconds_since(t0);
            while (nxt < count && t[nxt] <= now) ++nxt;
            bool progressed = false;
            for (auto& s : slots) {
                if (!s.busy) continue;
                if (s.early_busy) {
                    e = hipEventQuery(s.early);
                    if (e == hipSuccess) {
                        retire(s.early_rids);
                        s.early_busy = false;
                        progressed = true;
                    } else if (e != hipErrorNotReady) {
                        rc = hip_error(e, "hipEventQuery");
                        break;
                    }
                }
                e = hipEventQuery(s.done);
                if (e == hipErrorNotReady) continue;
                if (e != hipSuccess) {
                    rc = hip_error(e, "hipEventQuery");
                    break;
                }
                if (s.early_busy) retire(s.early_rids);
                retire(s.rids);
                s.busy = s.early_busy = false;
                progressed = true;
            }
            if (rc != FFT_OK) break;
            // waiting requests are spread over the free slots (a step takes its
            // share, rounded up), so that at low load requests run on separate
            // streams instead of one after another in one step
            int free_slots = 0;
            for (auto& x : slots) free_slots += x.busy ? 0 : 1;
            const size_t first_free = first_slot;
            for (size_t j = 0; j < slots.size(); ++j) {
                const size_t si = (first_free + j) % slots.size();
                Slot& s = slots[si];
                if (s.busy || head >= nxt) continue;
                size_t infl2 = inflight;
                const int64_t share = (nxt - head + free_slots - 1) / std::max(free_slots, 1);
                --free_slots;
                head = serve_admit(tr, order.data(), nxt, head, inflight, c, take, &infl2, share);
                if (take.empty()) continue;
                inflight = infl2;
                // placement per precision in admission order; split transforms
                // form their own group when they run through their plans
                const bool direct = (int64_t)take.size() <= c.direct_max;
                int64_t used[2] = {0, 0};
                uint64_t gen_first[2] = {0, 0};
                for (int d = 0; d < 2; ++d) {
                    whole[d].clear();
                    split[d].clear();
                }
                for (int64_t r : take) {
                    const int d = dt_index(dtype[r]);
                    if (used[d] == 0) gen_first[d] = first[r];
                    Group& g = c.split_direct && is_split(n[r], dtype[r]) ? split[d] : whole[d];
                    g.add(r, n[r], batch[r], used[d]);
                    used[d] += n[r] * batch[r];
                }
                // the step's requests of one precision are consecutive in that
                // precision's arrival order: one generator launch covers them
                for (int d = 0; d < 2 && rc == FFT_OK; ++d) {
                    if (used[d] && (e = fill_normal(d == 0 ? DT_F16 : DT_F32, s.arena[d], used[d], gen_first[d], c.seed,
                                                    s.st)) != hipSuccess)
                        rc = hip_error(e, "launch(fill)");
                }
                // one group's transforms: cached plans (two-pass ones on the
                // slot's workspace) or the slot's kernels; then the optional
                // output copies
                auto run_group = [&](Group* gs, bool plans_only) {
                    for (int d = 0; d < 2 && rc == FFT_OK; ++d) {
                        const Group& g = gs[d];
                        if (g.rid.empty()) continue;
                        const int dt = d == 0 ? DT_F16 : DT_F32;
                        if (plans_only) {
                            for (size_t i = 0; i < g.rid.size() && rc == FFT_OK; ++i) {
                                // plans per shape; a two-pass plan runs on this
                                // slot's workspace (launches on the slot's stream
                                // are ordered, other slots have their own)
                                fft_plan* p = plans.get(g.n[i], g.b[i], dt, 0);
                                if (!p) {
                                    rc = FFT_ENOMEM;
                                    break;
                                }
                                char* ptr = (char*)s.arena[d] + (size_t)g.off[i] * ebytes(dt);
                                if (p->k2) {
                                    rc = check_execute_args(p, ptr, ptr);
                                    if (rc == FFT_OK) rc = launch_plan_ws(p, ptr, ptr, s.st, plans.ws[si], p->chunk);
                                } else {
                                    rc = plan_execute(p, ptr, ptr, s.st);
                                }
                            }
                        } else {
                            rc = fft_serve_slot_launch(s.native[d], g.n.data(), g.b.data(), g.off.data(),
                                                       (int64_t)g.rid.size(), s.arena[d], s.st);
                        }
                        if (rc != FFT_OK || !out_dev || !out_off) continue;
                        for (size_t i = 0; i < g.rid.size(); ++i) {
                            const int64_t r = g.rid[i];
                            const size_t len = (size_t)n[r] * batch[r] * ebytes(dt);
                            if ((e = hipMemcpyAsync((char*)out_dev + out_off[r], (char*)s.arena[d] + (size_t)g.off[i] * ebytes(dt),
                                                    len, hipMemcpyDeviceToDevice, s.st)) != hipSuccess) {
                                rc = hip_error(e, "hipMemcpyAsync(output)");
                                break;
                            }
                        }
                    }
                };
                run_group(whole, direct);
                s.rids.clear();
                s.early_rids.clear();
                const bool two = (!whole[0].rid.empty() || !whole[1].rid.empty()) &&
                                 (!split[0].rid.empty() || !split[1].rid.empty());
                for (int d = 0; d < 2; ++d) {
                    std::vector<int64_t>& dst = two ? s.early_rids : s.rids;
                    dst.insert(dst.end(), whole[d].rid.begin(), whole[d].rid.end());
                    s.rids.insert(s.rids.end(), split[d].rid.begin(), split[d].rid.end());
                }
                if (rc == FFT_OK && two && (e = hipEventRecord(s.early, s.st)) != hipSuccess)
                    rc = hip_error(e, "hipEventRecord");
                if (rc == FFT_OK) run_group(split, true);
                if (rc != FFT_OK) break;
                if ((e = hipEventRecord(s.done, s.st)) != hipSuccess) {
                    rc = hip_error(e, "hipEventRecord");
                    break;
                }
                s.busy = true;
                s.early_busy = two;
                first_slot = (si + 1) % slots.size();
                st.steps += 1;
                st.direct_steps += direct ? 1 : 0;
                sum_req += (double)take.size();
                st.max_inflight_bytes = std::max<uint64_t>(st.max_inflight_bytes, inflight);
                int busy = 0;
                for (auto& x : slots) busy += x.busy ? 1 : 0;
                st.max_concurrent = std::max(st.max_concurrent, busy);
                progressed = true;
            }
            if (rc != FFT_OK) break;
            if (head < nxt && !progressed) {
                bool any = false;
                for (auto& x : slots) any |= x.busy;
                if (!any) rc = set_error(FFT_EINVAL, "a request exceeds the budget or a slot's capacity");
            }
        }
        st.mean_requests_per_step = st.steps ? sum_req / (double)st.steps : 0.0;
        cleanup();
        if (rc != FFT_OK) return rc;
    } else {
        // one launch per request, round-robin over the streams
        const int K = c.slots;
        std::vector<hipStream_t> sts(K, nullptr);
        std::vector<Ring> rings(K);
        const size_t ring = std::max<size_t>(c.slot_bytes, (max_req + 255) & ~size_t(255));
        int rc = FFT_OK;
        auto cleanup = [&]() {
            for (int k = 0; k < K; ++k) {
                if (sts[k]) (void)hipStreamSynchronize(sts[k]);
                if (rings[k].base) (void)hipFree(rings[k].base);
                if (sts[k]) (void)hipStreamDestroy(sts[k]);
            }
            for (void* w : plans.ws) (void)hipFree(w);
            plans.ws.clear();
        };
        for (int k = 0; k < K; ++k) {
            if ((e = hipStreamCreate(&sts[k])) != hipSuccess) {
                cleanup();
                return hip_error(e, "hipStreamCreate");
            }
            if ((e = hipMalloc((void**)&rings[k].base, ring)) != hipSuccess) {
                cleanup();
                return set_error(e == hipErrorOutOfMemory ? FFT_ENOMEM : FFT_EHIP, "request ring allocation failed");
            }
            rings[k].cap = ring;
            void* w = nullptr;
            if ((e = hipMalloc(&w, kMaxWorkspaceBytes)) != hipSuccess) {
                cleanup();
                return set_error(e == hipErrorOutOfMemory ? FFT_ENOMEM : FFT_EHIP, "workspace allocation failed");
            }
            plans.ws.push_back(w);
        }
        if ((e = hipDeviceSynchronize()) != hipSuccess) {
            cleanup();
            return hip_error(e, "hipDeviceSynchronize");
        }
        std::vector<std::deque<Inflight>> q(K);
        int64_t nxt = 0, completed = 0, k_rr = 0;
        size_t inflight = 0;
        const Clock::time_point t0 = Clock::now();
        while (completed < count && rc == FFT_OK) {
            const double now = seconds_since(t0);
            bool progressed = false;
            while (nxt < count && t[nxt] <= now) {
                const int64_t r = nxt;
                const int dt = dtype[r];
                const size_t len = (size_t)n[r] * batch[r] * ebytes(dt);
                if (inflight > 0 && inflight + 2 * len > c.budget_bytes) break;
                const int k = (int)(k_rr % K);
                size_t off = 0;
                if (!rings[k].alloc(len, &off)) break;          // wait for this stream's earlier requests
                ++k_rr;
                char* ptr = rings[k].base + off;
                fft_plan* p = plans.get(n[r], batch[r], dt, k);  // one plan per stream (two-pass workspaces)
                hipEvent_t ev = nullptr;
                if (!p) {
                    rc = FFT_ENOMEM;
                    break;
                }
                if ((e = fill_normal(dt, ptr, n[r] * batch[r], first[r], c.seed, sts[k])) != hipSuccess) {
                    rc = hip_error(e, "launch(fill)");
                    break;
                }
                if ((rc = plan_execute(p, ptr, ptr, sts[k])) != FFT_OK) break;
                if (out_dev && out_off &&
                    (e = hipMemcpyAsync((char*)out_dev + out_off[r], ptr, len, hipMemcpyDeviceToDevice, sts[k])) != hipSuccess) {
                    rc = hip_error(e, "hipMemcpyAsync(output)");
                    break;
                }
                if ((e = events.get(&ev)) != hipSuccess || (e = hipEventRecord(ev, sts[k])) != hipSuccess) {
                    rc = hip_error(e, "event");
                    break;
                }
                q[k].push_back(Inflight{r, ev, k, off, len});
                inflight += 2 * len;
                st.max_inflight_bytes = std::max<uint64_t>(st.max_inflight_bytes, inflight);
                ++nxt;
                progressed = true;
            }
            if (rc != FFT_OK) break;
            for (int k = 0; k < K && rc == FFT_OK; ++k) {
                while (!q[k].empty()) {
                    e = hipEventQuery(q[k].front().ev);
                    if (e == hipErrorNotReady) break;
                    if (e != hipSuccess) {
                        rc = hip_error(e, "hipEventQuery");
                        break;
                    }
                    const Inflight f = q[k].front();
                    q[k].pop_front();
                    done_t[f.rid] = seconds_since(t0);
                    inflight -= 2 * f.len;
                    rings[k].release_front();
                    events.put(f.ev);
                    ++completed;
                    progressed = true;
                }
            }
            (void)progressed;
        }
        st.steps = count;
        st.mean_requests_per_step = 1.0;
        cleanup();
        if (rc != FFT_OK) return rc;
    }
    double tmax = 0;
    for (int64_t r = 0; r < count; ++r) tmax = std::max(tmax, done_t[r]);
    st.wall_s = count ? tmax - t[0] : 0.0;
    if (stats) *stats = st;
    return FFT_OK;
}

}  // extern "C"
