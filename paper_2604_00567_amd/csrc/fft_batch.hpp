// Uneven-size batch: persistent, work-queue kernels run transforms of many
// sizes.  Work items are claimed in order with an atomic counter; each item
// is one workgroup's worth of units of one size class and runs the same
// register-pass / LDS-exchange code as the regular kernels.
//
// Transforms up to 2^14 points are single-unit items (whole transforms).
// Larger ones (2^15 .. 2^18) use the two-kernel split of the global schedule:
// column items (stages 1..log2 N1, into a workspace) and row items (the
// remaining stages, into the output).  The work list has two phases, each
// run by one launch of the persistent kernel: phase 0 = every column item,
// then the single-unit items; phase 1 = every row item.  The launch boundary
// is what makes the column results visible to the row items.  (Inside one
// launch, a row item would have to wait on counters with agent-scope
// acquire/release: on a part with one L2 per XCD each such release writes
// back and each acquire invalidates the whole L2 of its XCD, which cost far
// more than a second launch.)
#pragma once

#include "batch_launch.hpp"
#include "fft_device.hpp"
#include "tables.hpp"

namespace dsfft {

constexpr int kBatchThreads = kHostBatchThreads;
constexpr int kBatchMaxElems = 32;     // elements per lane, largest configuration
// Table entries [0, T) sit in LDS below the exchange area, copied once per
// workgroup of the persistent kernel: every pass after the first whose
// entries lie below T (binary16, T = 1024: all of them up to 2^10 points,
// the middle passes beyond, the column items' second pass; binary32, whose
// exchange leaves less room, T = 512) reads its twiddles there instead of
// through the vector memory path, where the lanes of a workgroup fetched the
// same entries again and again.
template <class E>
constexpr int batch_twiddle_prefix() {
    return sizeof(E) == 4 ? 1024 : 512;
}
static_assert(batch_twiddle_prefix<uint32_t>() <= kMinTableEntries, "the prefix lies inside every device table");
template <class E>
constexpr size_t batch_prefix_bytes() {
    return (size_t)batch_twiddle_prefix<E>() * sizeof(typename TwOf<E>::type);
}

// Work item (layout in batch_launch.hpp):
//   cfg        configuration id (HostBatchCfg), one compiled unit configuration
//   nunits     units in this item
//   first      single-unit items: first index into the offset list;
//              column/row items: first residue / row
//   log_m      column/row items: log2(N / NU)
//   phase      0 (columns, single-unit) or 1 (rows)
//   slot       column/row items: index of the large transform, else -1
//   in_off     column items: transform start in the input; row items: in the workspace
//   out_off    column items: transform start in the workspace; row items: in the output
using BatchItem = HostBatchItem;

// Unit geometry of one work item (TPX: the LDS table prefix).
template <int TPX>
struct BatchGeo {
    // no twiddle prefetch: the kernel's registers are the largest over all its
    // configurations, and prefetching raises that maximum into spills
    static constexpr bool kTwiddlePrefetch = false;
    static constexpr int kTwiddleLds = 0;
    static constexpr int kTwiddlePrefix = TPX;
    static constexpr int kEncoding = ENC_TABLE;
    // an item's units need not be consecutive in memory
    static constexpr bool kBlockRsrc = false;
    const int64_t* offs;
    BatchItem it;
    int lane_id;       // threadIdx.x, made opaque per configuration (batch_unit)
    template <int LOG_NU, int MODE>
    __device__ __forceinline__ UnitGeom get(int ul) const {
        UnitGeom u;
        u.in_stride = u.out_stride = 1;
        u.q0 = 0;
        u.log_lb = 0;
        if (MODE == MODE_SMALL) {
            const int64_t b = ul < it.nunits ? offs[it.first + ul] : 0;
            u.base_in = u.base_out = b;
        } else if (MODE == MODE_COLS) {
            const int r0 = it.first + ul;
            u.base_in = it.in_off + r0;
            u.base_out = it.out_off + r0;
            u.in_stride = u.out_stride = int64_t(1) << it.log_m;
        } else {
            const int q0 = it.first + ul;
            u.q0 = q0;
            u.log_lb = it.log_m;
            u.base_in = it.in_off + ((int64_t)q0 << LOG_NU);
            u.base_out = it.out_off + q0;
            u.out_stride = int64_t(1) << it.log_m;
        }
        return u;
    }
    __device__ __forceinline__ bool active(int ul) const { return ul < it.nunits; }
    __device__ __forceinline__ int tid() const { return lane_id; }
    __device__ __forceinline__ int64_t block_first(int) const { return 0; }
    __device__ __forceinline__ int64_t block_units(int) const { return 0; }
};

template <class E, int LOG_NU, int LOG_E, int UPW, int MODE, int LR0, int LR1, int LR2, class Geo>
__device__ __forceinline__ void batch_unit(E* lds, const typename TwOf<E>::type* __restrict__ lt,
                                           const E* src, E* dst, const Geo& geo) {
    static_assert((UPW << (LOG_NU - LOG_E)) == kBatchThreads, "batch configurations use 512 threads");
    static_assert((1 << LOG_E) <= kBatchMaxElems, "too many elements per lane");
    E v[1 << LOG_E];   // per configuration, so each case keeps its own registers
    // The thread index is read through an empty asm statement in each case:
    // index arithmetic common to several cases then cannot be hoisted above
    // the dispatch, where it would stay live in every case.
    Geo g = geo;
    g.lane_id = (int)threadIdx.x;
    asm volatile("" : "+v"(g.lane_id));
    unit_pass<E, LOG_NU, LOG_E, UPW, 1, MODE, LR0, LR1, LR2, 0, 0, 0, 0>(v, lds, lt, src, dst, g);
}

// Largest LDS footprint over the batch configurations, in elements.
constexpr int batch_lds_elems() {
    int m = 0;
    const int sizes[] = {
        512 * PassPlan<1, 1, 0, 0>::region(), 512 * PassPlan<2, 2, 0, 0>::region(),
        512 * PassPlan<3, 3, 0, 0>::region(), 128 * PassPlan<4, 2, 2, 0>::region(),
        128 * PassPlan<5, 3, 2, 0>::region(), 64 * PassPlan<6, 3, 3, 0>::region(),
        64 * PassPlan<7, 4, 3, 0>::region(), 32 * PassPlan<8, 4, 4, 0>::region(),
        32 * PassPlan<9, 5, 4, 0>::region(), 16 * PassPlan<10, 5, 5, 0>::region(),
        8 * PassPlan<11, 5, 3, 3>::region(), 2 * PassPlan<12, 4, 4, 4>::region(),
        2 * PassPlan<13, 5, 4, 4>::region(), 8 * PassPlan<10, 4, 3, 3>::region(),
        4 * PassPlan<12, 5, 4, 3>::region(), 64 * PassPlan<7, 4, 3, 0>::region(),
        64 * PassPlan<8, 5, 3, 0>::region(), 32 * PassPlan<9, 5, 4, 0>::region(),
        1 * PassPlan<14, 5, 5, 4>::region(), 32 * PassPlan<7, 3, 2, 2>::region(),
        16 * PassPlan<8, 3, 3, 2>::region(), 16 * PassPlan<9, 4, 3, 2>::region(),
        4 * PassPlan<11, 4, 4, 3>::region()};
    for (int s : sizes) m = s > m ? s : m;
    return m;
}

template <class E, class Geo>
__device__ __forceinline__ void batch_dispatch(int cfg, E* lds,
                                               const typename TwOf<E>::type* __restrict__ lt,
                                               const E* in, E* out, E* ws, const Geo& g) {
    switch (cfg) {
        case HB_N2: batch_unit<E, 1, 1, 512, MODE_SMALL, 1, 0, 0>(lds, lt, in, out, g); break;
        case HB_N4: batch_unit<E, 2, 2, 512, MODE_SMALL, 2, 0, 0>(lds, lt, in, out, g); break;
        case HB_N8: batch_unit<E, 3, 3, 512, MODE_SMALL, 3, 0, 0>(lds, lt, in, out, g); break;
        case HB_N16: batch_unit<E, 4, 2, 128, MODE_SMALL, 2, 2, 0>(lds, lt, in, out, g); break;
        case HB_N32: batch_unit<E, 5, 3, 128, MODE_SMALL, 3, 2, 0>(lds, lt, in, out, g); break;
        case HB_N64: batch_unit<E, 6, 3, 64, MODE_SMALL, 3, 3, 0>(lds, lt, in, out, g); break;
        case HB_N128: batch_unit<E, 7, 4, 64, MODE_SMALL, 4, 3, 0>(lds, lt, in, out, g); break;
        case HB_N256: batch_unit<E, 8, 4, 32, MODE_SMALL, 4, 4, 0>(lds, lt, in, out, g); break;
        case HB_N512: batch_unit<E, 9, 5, 32, MODE_SMALL, 5, 4, 0>(lds, lt, in, out, g); break;
        case HB_N1024: batch_unit<E, 10, 5, 16, MODE_SMALL, 5, 5, 0>(lds, lt, in, out, g); break;
        case HB_N2048: batch_unit<E, 11, 5, 8, MODE_SMALL, 5, 3, 3>(lds, lt, in, out, g); break;
        case HB_N4096: batch_unit<E, 12, 4, 2, MODE_SMALL, 4, 4, 4>(lds, lt, in, out, g); break;
        case HB_N8192: batch_unit<E, 13, 5, 2, MODE_SMALL, 5, 4, 4>(lds, lt, in, out, g); break;
        case HB_N1024_B: batch_unit<E, 10, 4, 8, MODE_SMALL, 4, 3, 3>(lds, lt, in, out, g); break;
        case HB_N4096_B: batch_unit<E, 12, 5, 4, MODE_SMALL, 5, 4, 3>(lds, lt, in, out, g); break;
        case HB_ROWS128: batch_unit<E, 7, 4, 64, MODE_ROWS, 4, 3, 0>(lds, lt, ws, out, g); break;
        case HB_COLS256: batch_unit<E, 8, 5, 64, MODE_COLS, 5, 3, 0>(lds, lt, in, ws, g); break;
        case HB_ROWS256: batch_unit<E, 8, 5, 64, MODE_ROWS, 5, 3, 0>(lds, lt, ws, out, g); break;
        case HB_COLS512: batch_unit<E, 9, 5, 32, MODE_COLS, 5, 4, 0>(lds, lt, in, ws, g); break;
        case HB_ROWS512: batch_unit<E, 9, 5, 32, MODE_ROWS, 5, 4, 0>(lds, lt, ws, out, g); break;
        case HB_N16384: batch_unit<E, 14, 5, 1, MODE_SMALL, 5, 5, 4>(lds, lt, in, out, g); break;
        case HB_N128_B: batch_unit<E, 7, 3, 32, MODE_SMALL, 3, 2, 2>(lds, lt, in, out, g); break;
        case HB_N256_B: batch_unit<E, 8, 3, 16, MODE_SMALL, 3, 3, 2>(lds, lt, in, out, g); break;
        case HB_N512_B: batch_unit<E, 9, 4, 16, MODE_SMALL, 4, 3, 2>(lds, lt, in, out, g); break;
        case HB_N2048_B: batch_unit<E, 11, 4, 4, MODE_SMALL, 4, 4, 3>(lds, lt, in, out, g); break;
        default: break;
    }
}

// Whole transforms too large for the batch kernel's LDS (binary16, 2^15 and
// 2^16 points) run in a kernel of their own, one transform per workgroup,
// with unit u of the launch at element offset offs[u]; table entries [0, TPX)
// sit in LDS below the exchange area (the middle pass reads them there).
template <int TPX>
struct ListGeo {
    static constexpr bool kTwiddlePrefetch = false;
    static constexpr int kTwiddleLds = 0;
    static constexpr int kTwiddlePrefix = TPX;
    static constexpr int kEncoding = ENC_TABLE;
    // one unit per workgroup (the transform at offs[ublk])
    static constexpr bool kBlockRsrc = true;
    const int64_t* offs;
    int64_t ublk, units;
    int lane_id;
    template <int LOG_NU, int MODE>
    __device__ __forceinline__ UnitGeom get(int ul) const {
        UnitGeom u;
        u.in_stride = u.out_stride = 1;
        u.q0 = 0;
        u.log_lb = 0;
        u.base_in = u.base_out = (ublk + ul < units) ? offs[ublk + ul] : 0;
        return u;
    }
    __device__ __forceinline__ bool active(int ul) const { return ublk + ul < units; }
    __device__ __forceinline__ int tid() const { return lane_id; }
    __device__ __forceinline__ int64_t block_first(int) const { return ublk < units ? offs[ublk] : 0; }
    __device__ __forceinline__ int64_t block_units(int) const { return ublk < units ? 1 : 0; }
};

template <class E, int LOG_NU, int LOG_E, int LR0, int LR1, int LR2, int TPX>
__global__ void __launch_bounds__(1 << (LOG_NU - LOG_E))
fft_list_kernel(const E* in, E* out, const typename TwOf<E>::type* __restrict__ lt,
                const int64_t* __restrict__ offs, int64_t count) {
    using TW = typename TwOf<E>::type;
    static_assert(TPX <= kMinTableEntries, "the prefix lies inside every device table");
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    // the first exchange's barrier orders the copy before the middle pass
    copy_table_prefix<TW, TPX, (1 << (LOG_NU - LOG_E))>(lt, lds_raw);
    E* lds = reinterpret_cast<E*>(lds_raw + (size_t)TPX * sizeof(TW));
    E v[1 << LOG_E];
    const ListGeo<TPX> gp{offs, (int64_t)blockIdx.x, count, (int)threadIdx.x};
    unit_pass<E, LOG_NU, LOG_E, 1, 1, MODE_SMALL, LR0, LR1, LR2, 0, 0, 0, 0>(v, lds, lt, in, out, gp);
}

// Items first .. first + nitems - 1 of one phase.  q[0] is the phase's queue
// head and q[1] counts the workgroups that have left the loop; both are zero
// at launch, and the last workgroup to leave sets them back to zero for the
// next launch on the stream (so no clearing launch is needed).
template <class E>
__global__ void __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(sizeof(E) == 4 ? 4 : 2)))
fft_batch_kernel(const E* in, E* out, E* ws, const typename TwOf<E>::type* __restrict__ lt,
                 const BatchItem* __restrict__ items, const int64_t* __restrict__ offs,
                 int first, int nitems, unsigned* q) {
    unsigned* head = q;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    // the barrier after the first claim publishes the copy
    copy_table_prefix<typename TwOf<E>::type, batch_twiddle_prefix<E>(), kBatchThreads>(lt, lds_raw);
    E* lds = reinterpret_cast<E*>(lds_raw + batch_prefix_bytes<E>());
    // Claims run one item ahead: the claim of the next item is issued when
    // the current one starts, so its round trip overlaps the current item's
    // work, and published in LDS when the item ends.  Two slots alternate:
    // the slot written at the end of item k was last read after the barrier
    // that ended item k - 2, and every thread has since passed the barrier
    // that ended item k - 1.
    __shared__ int s_item[2];
    if (threadIdx.x == 0) s_item[0] = (int)atomicAdd(head, 1u);
    __syncthreads();
    // the item index is uniform: in scalar registers, the item's fields and
    // the addresses derived from them stay scalar too
    int idx = __builtin_amdgcn_readfirstlane(s_item[0]);
    for (int k = 1; idx < nitems; ++k) {
        // the returned index is needed only at the end of the item
        const unsigned next = threadIdx.x == 0 ? atomicAdd(head, 1u) : 0u;
        const BatchItem it = items[first + idx];
        const BatchGeo<batch_twiddle_prefix<E>()> geo{offs, it, 0};
        // An opaque copy of the table pointer per item keeps each case's
        // twiddle address arithmetic inside the loop; hoisted out of it, the
        // addresses of every case would stay live across the whole loop.
        const typename TwOf<E>::type* lt_item = lt;
        asm volatile("" : "+s"(lt_item));
        batch_dispatch<E>(it.cfg, lds, lt_item, in, out, ws, geo);
        if (threadIdx.x == 0) s_item[k & 1] = (int)next;
        __syncthreads();   // LDS consumed before the next item reuses it; next claim visible
        idx = __builtin_amdgcn_readfirstlane(s_item[k & 1]);
    }
    // This workgroup's claims are over (its last one returned an index past
    // the end).  The last workgroup out sees every claim made and resets.
    if (threadIdx.x == 0 && atomicAdd(&q[1], 1u) == gridDim.x - 1) {
        atomicExch(&q[0], 0u);
        atomicExch(&q[1], 0u);
    }
}

}  // namespace dsfft
