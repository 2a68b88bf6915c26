// HIP kernels and C-ABI entry points of liblbessel (gfx950, wave64).
//
// Grouped kernel (every public forward / derivative / vMF call):
//   one workgroup = 256 threads = 4 wavefronts owns a tile of 1024
//   consecutive elements (4 per thread; two evaluations per element, orders
//   v and v + 1, for the derivatives and the vMF gradient).
//   1. coalesced loads of (v, x); special values are resolved at once; every
//      other evaluation gets its class from its own (v, x): branch, Debye
//      term-count tier, fallback cost bucket;
//   2. per class present in a wavefront, ballots + popcounts give per-wave
//      counts.  A tile with a single class evaluates its elements in place
//      (coalesced, no list); otherwise one short scan turns the counts into
//      offsets of a class-sorted list in LDS (fallback buckets, costliest
//      first, then the Debye tiers, then Hankel);
//   3. the list is cut into 64-entry chunks that the wavefronts take from an
//      LDS counter, so a wavefront runs one class except in the chunks that
//      straddle two, and expensive chunks spread over the four wavefronts;
//   4. results go straight to HBM, or (one-order K, and I in binary32, whose
//      pairs are staged in LDS) into LDS and out in one coalesced store, or
//      into LDS to be combined per element (two orders per element).
// The branch of an evaluation depends only on its own (v, x), never on its
// neighbours, so the grouped and the ungrouped kernel give the same bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include <hipcub/hipcub.hpp>

#include "lbessel.h"
#include "lbessel_serve.h"
#include "lbessel_device.hpp"

namespace lbessel {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Operation applied around the log-Bessel evaluation(s) of one element.
enum : int {
    OP_LOG = 0,       // out = log B_v(x)
    OP_GRAD = 1,      // out = g * d/dx log B_v(x) from orders v and v + 1
    OP_VMF = 2,       // out = (p/2-1) log k - (p/2) log 2pi - log I_{p/2-1}(k)
    OP_VMF_GRAD = 3,  // out = -exp(log I_{p/2}(k) - log I_{p/2-1}(k))
};

template <int OP> struct OpTraits {
    static constexpr int nv = (OP == OP_GRAD || OP == OP_VMF_GRAD) ? 2 : 1;
    static constexpr bool scalar_order = (OP == OP_VMF || OP == OP_VMF_GRAD);
};

// Kernel arguments.  For the vMF operations v is unused, the order is the
// scalar vs = p/2 - 1 and x holds kappa.
template <typename T> struct Args {
    const T *v;
    const T *x;
    const T *g;     // upstream gradient (OP_GRAD) or nullptr
    T *out;
    int64_t n;
    T vs;           // scalar order (vMF)
    T p;            // vMF dimension
};

template <typename T, int KIND, int OP>
__device__ __forceinline__ T order_of(const Args<T> &a, int64_t i) {
    if (OpTraits<OP>::scalar_order)
        return a.vs;
    if (a.v == nullptr)   // one order for the whole array (uniform branch)
        return (KIND == KIND_K) ? fabs(a.vs) : a.vs;
    const T v = a.v[i];
    return (KIND == KIND_K) ? fabs(v) : v;
}

// Elements whose final result is a limit that needs no evaluation.
template <typename T, int KIND, int OP>
__device__ __forceinline__ bool element_special(T v, T x, T g, T p, T *res) {
    const T inf = __builtin_huge_val();
    const T nan = __builtin_nan("");
    if (OP == OP_LOG) {
        return special_value<T, KIND>(v, x, res);
    } else if (OP == OP_GRAD) {
        if (KIND == KIND_I) {
            if (!(v >= T(0)) || !(x >= T(0)) || v == inf) { *res = nan; return true; }
            if (x == T(0)) { *res = g * ((v == T(0)) ? T(0) : inf); return true; }
            if (x == inf) { *res = g; return true; }
        } else {
            if (!(x >= T(0)) || v != v || v == inf) { *res = nan; return true; }
            if (x == T(0)) { *res = -g * inf; return true; }
            if (x == inf) { *res = -g; return true; }
        }
        return false;
    } else if (OP == OP_VMF) {
        if (!(x >= T(0)) || x == inf) { *res = nan; return true; }
        if (x == T(0)) {
            *res = v * Cst<T>::ln2 + lgamma(v + T(1)) - T(0.5) * p * Cst<T>::log_2pi;
            return true;
        }
        return false;
    } else {  // OP_VMF_GRAD
        if (!(x >= T(0)) || x == inf) { *res = nan; return true; }
        if (x == T(0)) { *res = T(0); return true; }
        return false;
    }
}

template <typename T, int KIND, int OP>
__device__ __forceinline__ T combine(T v, T x, T g, T p, T y0, T y1) {
    if (OP == OP_LOG)
        return y0;
    if (OP == OP_GRAD)
        return (KIND == KIND_I) ? g * (exp(y1 - y0) + v / x) : g * (v / x - exp(y1 - y0));
    if (OP == OP_VMF)
        return v * log(x) - T(0.5) * p * Cst<T>::log_2pi - y0;
    return -exp(y1 - y0);  // OP_VMF_GRAD
}

// One evaluation that may still hit a special value (the v + 1 order).
template <typename T, int KIND, int VAR = VAR_DEFAULT>
__device__ __forceinline__ T eval_full(T v, T x, const FbTab<KIND, T> *kt) {
    T y;
    if (special_value<T, KIND>(v, x, &y))
        return y;
    return eval_branch<T, KIND, VAR>(classify_var<T, KIND, VAR>(v, x), v, x, kt);
}

// LDS copy of the fallback's tables (K: e^{+-t}; I: log Gamma(1 + v)), loaded
// by every workgroup before its first evaluation (all threads must reach the
// call).
template <int KIND, typename T>
__device__ __forceinline__ FbTab<KIND, T> *fb_tab_storage() {
    __shared__ FbTab<KIND, T> kt;
    return &kt;
}

template <int KIND, typename T>
__device__ __forceinline__ void fb_tab_load(FbTab<KIND, T> *kt) {
    if constexpr (KIND == KIND_K)
        ktab_load(kt);
    else
        lgtab_load(kt);
}

template <int KIND, typename T>
__device__ __forceinline__ const FbTab<KIND, T> *ktab_for_kind() {
    FbTab<KIND, T> *kt = fb_tab_storage<KIND, T>();
    fb_tab_load<KIND, T>(kt);
    return kt;
}

// ---------------------------------------------------------------------------
// Ungrouped kernel: one element per thread, no regrouping.
// ---------------------------------------------------------------------------
template <typename T, int KIND, int OP, int VAR = VAR_DEFAULT>
__global__ __launch_bounds__(kThreads) void k_ungrouped(Args<T> a) {
    const auto *kt = ktab_for_kind<KIND, T>();
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= a.n)
        return;
    const T v = order_of<T, KIND, OP>(a, i);
    const T x = a.x[i];
    const T g = (a.g != nullptr) ? a.g[i] : T(1);
    T res;
    if (element_special<T, KIND, OP>(v, x, g, a.p, &res)) {
        a.out[i] = res;
        return;
    }
    const T y0 = eval_full<T, KIND, VAR>(v, x, kt);
    const T y1 = (OpTraits<OP>::nv == 2) ? eval_full<T, KIND, VAR>(v + T(1), x, kt) : y0;
    a.out[i] = combine<T, KIND, OP>(v, x, g, a.p, y0, y1);
}

// ---------------------------------------------------------------------------
// Grouped kernel
// ---------------------------------------------------------------------------
template <int NV, int NTH = kThreads> struct TileCfg {
    static constexpr int ept = 4;                        // elements per thread
    static constexpr int tile = NTH * ept;               // elements per tile
    static constexpr int slots = ept * NV;               // evaluations per thread
};

// Classes an evaluation is sorted into inside a tile: Hankel, Debye and the
// fallback (three classes for the two-order operations).  The fallbacks'
// costs vary ~10x with (v, x):
// the K integral's node count and the I series' term count.  For the
// one-order operations the fallback is therefore split into buckets by an
// estimate of that count (kKBuckets for K: six by node count and one for the
// interior windows; in the default variant four by Temme-series cost and one
// for the integral; kIBuckets for I), so the lanes of one 64-entry chunk run
// loops of similar length.  List order: costliest
// bucket first, then the cheaper ones, Debye, Hankel.
// The Debye class is split the same way into its term-count tiers (U_13,
// U_9, U_6, U_4; u_tier), which differ ~2x in cost.
// Class ids: 0 = Hankel, 1..ub = Debye tier, 1+ub.. = fallback bucket.
constexpr int kKBuckets = 7;
constexpr int kIBuckets = 4;
template <int KIND, int OP, int VAR> struct Classes {
    static constexpr bool one = (OpTraits<OP>::nv == 1);
    static constexpr int fb =
        !one ? 1
        : (KIND == KIND_K) ? ((VAR == VAR_DEFAULT || VAR == VAR_PAPER_REGIMES) ? kKBuckets : 1)
                           : kIBuckets;
    static constexpr int ub = (one && VAR == VAR_DEFAULT) ? kUTiers : 1;
    static constexpr int u0 = 1;          // first Debye class
    static constexpr int f0 = 1 + ub;     // first fallback class
    static constexpr int n = 1 + ub + fb;
    static constexpr int bits = (n > 15) ? 5 : (n > 3) ? 4 : 2;
    static constexpr int none = (1 << bits) - 1;
};

// Workgroup size of a grouped kernel.  The one-order K kernels run 512
// threads on 2048-element tiles: their fallback elements (~40% of a mixed
// launch) differ ~10x in cost, and the longer each class-sorted list, the
// fewer of its 64-lane chunks straddle two cost classes (2^26-pair stress
// grid: 3.15 -> 2.95 ms against 1024-element tiles; 4096-element tiles gain
// little more there and lose on launches of one class, whose 16-wave
// workgroups wait at the tile barrier with little else to overlap).  Their
// LDS grows with the tile (16 bytes of staging per element): four
// workgroups per CU, 32 waves.  Binary64 only: the binary32 K kernels are
// ~2% faster on 1024-element tiles (stress grid 0.81-0.83 -> 0.80 ms, the
// per-order sets ~1%), as are the other kernels, which keep 256 threads.
#ifndef LBESSEL_K_THREADS
#define LBESSEL_K_THREADS 512
#endif
template <typename T, int KIND, int OP, int VAR> struct GroupShape {
    static constexpr int threads =
        (KIND == KIND_K && sizeof(T) == 8 && OpTraits<OP>::nv == 1 &&
         (VAR == VAR_DEFAULT || VAR == VAR_PAPER_REGIMES))
            ? LBESSEL_K_THREADS
            : kThreads;
    // LDS-bound at 4 (or 2) workgroups per CU: 8 waves per SIMD (<= 64 VGPRs)
    static constexpr int waves_per_eu = (threads > kThreads) ? 8 : 1;
};

// One-order operations of K, and of I in binary32 (STAGE): the tile's (order,
// argument) pairs are staged in LDS in step 1 and the results in the order
// slots in step 4, so HBM sees one coalesced read of (v, x) and one coalesced
// write of the results per element, however long the tile's integrals take,
// and step 4 reads its operands from LDS instead of waiting on L2.  The
// binary64 I kernels stage the arguments alone (XS): 16 KB of full staging
// would cut them from 8 workgroups per CU to 6, which costs more than the
// re-reads of the orders (stress grid 0.98-1.00 -> 0.95 ms with the
// arguments staged; 2-5% slower fully staged).  The two-order operations
// finish a tile quickly enough that the step-4 re-reads hit L2.
template <typename T, int NV, int NC, bool STAGE, int NTH, bool XS = false> struct Smem {
    using Cfg = TileCfg<NV, NTH>;
    static constexpr int NW = NTH / 64;
    T sv[STAGE ? Cfg::tile : 1];                         // order, then result
    T sx[(STAGE || XS) ? Cfg::tile : 1];                 // argument
    uint16_t list[Cfg::tile * NV];                       // evaluation ids, class-sorted
    uint16_t cnt[NC][Cfg::slots][NW];                    // counts, then offsets
    int start[NC];                                       // first list position per class
    int n_fb, n_fb_u, n_all;                             // list segment ends
    uint32_t wmask[NW];                                  // classes present, per wave
    int chunk;                                           // next chunk to evaluate
    T res[(NV == 2) ? Cfg::tile * 2 : 1];                // log-values of both orders
};

__device__ __forceinline__ int rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
}

// One tile of NTH threads (workgroup-wide: every thread of the workgroup must
// call it).
template <typename T, int KIND, int OP, int VAR = VAR_DEFAULT, int NTH = kThreads>
__device__ __forceinline__ void grouped_tile(const Args<T> &a, int64_t tile) {
    static_assert(VAR != VAR_SEVEN, "the grouped kernel sorts three branches");
    constexpr int NV = OpTraits<OP>::nv;
    constexpr int EPT = TileCfg<NV, NTH>::ept;
    constexpr int TILE = TileCfg<NV, NTH>::tile;
    constexpr int SLOTS = TileCfg<NV, NTH>::slots;
    constexpr int NW = NTH / 64;
    using C = Classes<KIND, OP, VAR>;
    constexpr int NC = C::n;
    constexpr int BITS = C::bits;
    constexpr uint32_t MASK = (1u << BITS) - 1;
    static_assert(SLOTS * BITS <= 32, "class codes of one thread fit 32 bits");
    static_assert(NC < 32, "class masks fit 32 bits");
    static_assert(TILE * NV <= 65536, "evaluation ids fit 16 bits");
    constexpr bool STAGE = (NV == 1) && (KIND == KIND_K || sizeof(T) == 4);
    // binary64 log I stages the arguments alone (8 KB: still 8 workgroups
    // per CU), so step 4 re-reads only the orders from L2 or HBM
    constexpr bool XSTAGE = (NV == 1) && !STAGE && (VAR == VAR_DEFAULT);
    __shared__ Smem<T, NV, NC, STAGE, NTH, XSTAGE> sm;

    // the fallback's tables, loaded below only if the tile has fallback work
    FbTab<KIND, T> *kt = fb_tab_storage<KIND, T>();
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int64_t base = tile * TILE;

    // 1. load, screen, classify.  code: BITS bits per evaluation slot
    //    (slot = r * NV + sub), C::none = nothing to evaluate.
    uint32_t code = 0;
    uint32_t done = 0;   // bit r: element r finished in this step (or out of range)
    // unstaged kernels keep the loaded operands for a one-class tile, which
    // then evaluates without a second (L2) read; the measurement variants,
    // whose branch code needs more registers, read again instead (kept, the
    // operands would cost them a wave per SIMD)
    constexpr bool KEEP = (VAR == VAR_DEFAULT);
    T vr[EPT], xr[EPT];
#pragma unroll
    for (int r = 0; r < EPT; ++r) {
        const int e = r * NTH + tid;
        const int64_t i = base + e;
        int b0 = C::none, b1 = C::none;
        vr[r] = T(0);
        xr[r] = T(1);
        if (i >= a.n) {
            done |= 1u << r;
        } else {
            const T v = order_of<T, KIND, OP>(a, i);
            const T x = a.x[i];
            vr[r] = v;
            xr[r] = x;
            T res;
            const T g = (a.g != nullptr) ? a.g[i] : T(1);
            if (element_special<T, KIND, OP>(v, x, g, a.p, &res)) {
                a.out[i] = res;
                done |= 1u << r;
            } else if (NV == 1) {
                if (STAGE) {
                    sm.sv[e] = v;
                    sm.sx[e] = x;
                } else if (XSTAGE) {
                    sm.sx[e] = x;
                }
                const int br = classify_var<T, KIND, VAR>(v, x);
                if (br == BR_MU)
                    b0 = 0;
                else if (br == BR_U)
                    b0 = C::u0 + ((C::ub > 1) ? u_tier(v) : 0);
                else
                    b0 = C::f0 + ((C::fb == 1) ? 0
                                  : (KIND == KIND_K)
                                      ? k_cost_bucket<kKBuckets, VAR == VAR_DEFAULT>(double(v),
                                                                                     double(x))
                                                     : i_cost_bucket<kIBuckets>(x));
            } else {
                T ys;
                if (special_value<T, KIND>(v, x, &ys))
                    sm.res[e * 2] = ys;
                else
                    b0 = classify<T, KIND>(v, x);
                const T v1 = v + T(1);
                if (special_value<T, KIND>(v1, x, &ys))
                    sm.res[e * 2 + 1] = ys;
                else
                    b1 = classify<T, KIND>(v1, x);
            }
        }
        code |= uint32_t(b0) << (BITS * (r * NV));
        if (NV == 2)
            code |= uint32_t(b1) << (BITS * (r * NV + 1));
    }

    // 2. per-wave counts per (class, slot), then offsets within each class.
    //    Only the classes present in the wave take ballots (OR of the lanes'
    //    class masks); the others count 0.
    uint32_t present = 0;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s)
        present |= 1u << ((code >> (BITS * s)) & MASK);
    present &= ~(1u << C::none);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        present |= uint32_t(__shfl_xor(int(present), off));
    present = __builtin_amdgcn_readfirstlane(present);
    for (int c = lane; c < NC * SLOTS; c += 64)
        sm.cnt[c / SLOTS][c % SLOTS][wave] = 0;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int b = (code >> (BITS * s)) & MASK;
        for (uint32_t pm = present; pm != 0; pm &= pm - 1) {
            const int br = __builtin_ctz(pm);
            const uint64_t m = __ballot(b == br);
            if (lane == 0)
                sm.cnt[br][s][wave] = __popcll(m);
        }
    }
    if (lane == 0)
        sm.wmask[wave] = present;
    __syncthreads();

    // Uniform tile (one class only, e.g. one order whose arguments all fall
    // in one regime): every wave already runs one branch, so each thread
    // evaluates its own elements in input order, with coalesced loads and
    // stores, and the tile skips the scan and the list.  The value of an
    // element is the same either way.
    uint32_t tile_mask = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w)
        tile_mask |= sm.wmask[w];
    if (NV == 1 && (tile_mask & (tile_mask - 1)) == 0) {   // workgroup-uniform
        if (tile_mask == 0)
            return;   // every element was special or out of range (already stored)
        const int cls = __builtin_ctz(tile_mask);
        if (cls >= C::f0)
            fb_tab_load<KIND, T>(kt);
        const int b = (cls >= C::f0) ? BR_FB : (cls >= C::u0 ? BR_U : BR_MU);
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            if (done & (1u << r))
                continue;
            const int e = r * NTH + tid;
            const T v = STAGE ? sm.sv[e] : KEEP ? vr[r] : order_of<T, KIND, OP>(a, base + e);
            const T x = STAGE ? sm.sx[e] : KEEP ? xr[r] : a.x[base + e];
            const T y = eval_branch<T, KIND, VAR>(b, v, x, kt);
            a.out[base + e] = combine<T, KIND, OP>(v, x, T(1), a.p, y, y);
        }
        return;
    }

    if (tid < NC) {
        const int br = tid;
        int run = 0;
        for (int s = 0; s < SLOTS; ++s)
            for (int w = 0; w < NW; ++w) {
                const int c = sm.cnt[br][s][w];
                sm.cnt[br][s][w] = run;
                run += c;
            }
        sm.start[br] = run;   // class total for now
    }
    __syncthreads();
    if (tid == 0) {
        // list order: fallback buckets from costliest down, Debye tiers from
        // costliest (U_13) down, Hankel
        int pos = 0;
        for (int b = NC - 1; b >= C::f0; --b) {
            const int t = sm.start[b];
            sm.start[b] = pos;
            pos += t;
        }
        sm.n_fb = pos;
        for (int b = C::u0; b < C::f0; ++b) {
            const int t = sm.start[b];
            sm.start[b] = pos;
            pos += t;
        }
        sm.n_fb_u = pos;
        const int tm = sm.start[0];
        sm.start[0] = pos;
        sm.n_all = pos + tm;
        sm.chunk = 0;
    }
    __syncthreads();
    const int n_fb = sm.n_fb;                     // all fallback buckets
    const int n_fb_u = sm.n_fb_u;                 // ... plus Debye
    const int n_all = sm.n_all;
    if (n_fb > 0)                                 // workgroup-uniform
        fb_tab_load<KIND, T>(kt);

    // 3. scatter evaluation ids in list order
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int b = (code >> (BITS * s)) & MASK;
        for (uint32_t pm = present; pm != 0; pm &= pm - 1) {
            const int br = __builtin_ctz(pm);
            const uint64_t m = __ballot(b == br);
            if (b == br) {
                const int pos = sm.start[br] + sm.cnt[br][s][wave] + rank_below(m);
                const int r = s / NV, sub = s - (s / NV) * NV;
                sm.list[pos] = uint16_t((r * NTH + tid) * NV + sub);
            }
        }
    }
    __syncthreads();

    // 4. evaluate 64-entry chunks
    const int n_chunks = (n_all + 63) >> 6;
    for (;;) {
        int c = 0;
        if (lane == 0)
            c = atomicAdd(&sm.chunk, 1);
        c = __shfl(c, 0);
        if (c >= n_chunks)
            break;
        const int j = (c << 6) + lane;
        if (j < n_all) {
            const int id = sm.list[j];
            const int e = id / NV;
            const int sub = id - e * NV;
            const int b = (j < n_fb) ? BR_FB : (j < n_fb_u ? BR_U : BR_MU);
            if (STAGE) {
                sm.sv[e] = eval_branch<T, KIND, VAR>(b, sm.sv[e], sm.sx[e], kt);
            } else {
                const int64_t i = base + e;
                const T v = order_of<T, KIND, OP>(a, i);
                const T x = XSTAGE ? sm.sx[e] : a.x[i];
                const T y = eval_branch<T, KIND, VAR>(b, v + T(sub), x, kt);
                if (NV == 2)
                    sm.res[id] = y;
                else
                    a.out[i] = combine<T, KIND, OP>(v, x, T(1), a.p, y, y);
            }
        }
    }

    // 5a. staged operations: coalesced store of the results
    if (STAGE) {
        __syncthreads();
        const T vs = OpTraits<OP>::scalar_order ? a.vs : T(0);   // combine's order (vMF)
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            if (done & (1u << r))
                continue;
            const int e = r * NTH + tid;
            const T y = sm.sv[e];
            a.out[base + e] = combine<T, KIND, OP>(vs, sm.sx[e], T(1), a.p, y, y);
        }
        return;
    }

    // 5b. two-order operations: combine per element
    if (NV == 2) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            if (done & (1u << r))
                continue;
            const int e = r * NTH + tid;
            const int64_t i = base + e;
            const T v = order_of<T, KIND, OP>(a, i);
            const T x = a.x[i];
            const T g = (a.g != nullptr) ? a.g[i] : T(1);
            a.out[i] = combine<T, KIND, OP>(v, x, g, a.p, sm.res[e * 2], sm.res[e * 2 + 1]);
        }
    }
}

template <typename T, int KIND, int OP, int VAR = VAR_DEFAULT>
__global__ __launch_bounds__((GroupShape<T, KIND, OP, VAR>::threads))
__attribute__((amdgpu_waves_per_eu(GroupShape<T, KIND, OP, VAR>::waves_per_eu)))
void k_grouped(Args<T> a) {
    grouped_tile<T, KIND, OP, VAR, GroupShape<T, KIND, OP, VAR>::threads>(a, blockIdx.x);
}

// Launch of k_grouped over a.n elements with its workgroup size and tile.
template <typename T, int KIND, int OP, int VAR = VAR_DEFAULT>
int launch_grouped(const Args<T> &a, hipStream_t st) {
    constexpr int nth = GroupShape<T, KIND, OP, VAR>::threads;
    constexpr int tile = TileCfg<OpTraits<OP>::nv, nth>::tile;
    const int64_t b = (a.n + tile - 1) / tile;
    if (b > int64_t(0x7fffffff))
        return LBESSEL_EINVAL;
    hipLaunchKernelGGL((k_grouped<T, KIND, OP, VAR>), dim3(uint32_t(b)), dim3(nth), 0, st, a);
    return (hipGetLastError() == hipSuccess) ? LBESSEL_OK : LBESSEL_EHIP;
}

// ---------------------------------------------------------------------------
// Global sort by branch (the paper's GPU grouping), for measurement: keys
// from the classifier, a radix sort of (key, index) pairs, then one element
// per thread in sorted order, gathered by index and scattered back.
// ---------------------------------------------------------------------------
template <int KIND, int VAR>
__global__ __launch_bounds__(kThreads) void k_sort_keys(const double *__restrict__ v,
                                                        const double *__restrict__ x,
                                                        uint8_t *__restrict__ key,
                                                        uint32_t *__restrict__ idx, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n)
        return;
    const double vv = (KIND == KIND_K) ? fabs(v[i]) : v[i];
    double y;
    key[i] = special_value<double, KIND>(vv, x[i], &y) ? uint8_t(7)
                                                       : uint8_t(classify_var<double, KIND, VAR>(vv, x[i]));
    idx[i] = uint32_t(i);
}

template <int KIND, int VAR>
__global__ __launch_bounds__(kThreads) void k_sorted_eval(const uint8_t *__restrict__ key,
                                                          const uint32_t *__restrict__ idx,
                                                          const double *__restrict__ v,
                                                          const double *__restrict__ x,
                                                          double *__restrict__ out, int64_t n) {
    const auto *kt = ktab_for_kind<KIND, double>();
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t e = idx[i];
    const double vv = (KIND == KIND_K) ? fabs(v[e]) : v[e];
    const double xx = x[e];
    double y;
    if (key[i] == 7)
        special_value<double, KIND>(vv, xx, &y);
    else
        y = eval_branch<double, KIND, VAR>(int(key[i]), vv, xx, kt);
    out[e] = y;
}

// ---------------------------------------------------------------------------
// Segmented grouped kernel: many independent arrays in one launch (the
// serving runtime's batches).  Segment s owns the tiles from segs[s].tile0
// up to the next segment's tile0; each tile is the same grouped_tile as in
// the single-array kernel, so every result equals the single-array one.
// ---------------------------------------------------------------------------
// Tile blockIdx.x of a segmented launch over segs[0 .. nseg): segs is a
// device table or the kernel-argument copy of k_grouped_seg_inline.
template <typename T, int KIND, typename Segs>
__device__ __forceinline__ void seg_tile(const Segs &segs, int nseg) {
    const int64_t t = blockIdx.x;
    // largest s with segs[s].tile0 <= t (uniform across the workgroup)
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].tile0 <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    const lbessel_segment_t sg = segs[lo];
    if (t < sg.tile0)   // malformed table: leave the tile alone (workgroup-uniform)
        return;
    Args<T> a{static_cast<const T *>(sg.v), static_cast<const T *>(sg.x), nullptr,
              static_cast<T *>(sg.out), sg.n, T(0), T(0)};
    grouped_tile<T, KIND, OP_LOG>(a, t - sg.tile0);
}

template <typename T, int KIND>
__global__ __launch_bounds__(kThreads) void k_grouped_seg(
    const lbessel_segment_t *__restrict__ segs, int nseg) {
    seg_tile<T, KIND>(segs, nseg);
}

// The segment table passed by value in the kernel arguments (no device copy).
struct SegPack {
    lbessel_segment_t s[LBESSEL_SEG_INLINE_MAX];
    __device__ const lbessel_segment_t &operator[](int i) const { return s[i]; }
};

template <typename T, int KIND>
__global__ __launch_bounds__(kThreads) void k_grouped_seg_inline(SegPack pack, int nseg) {
    seg_tile<T, KIND>(pack, nseg);
}

// ---------------------------------------------------------------------------
// Orders 0 and 1: one element per thread, polynomial evaluations only
// ---------------------------------------------------------------------------
template <typename T, int KIND, int V>
__global__ __launch_bounds__(kThreads) void k_order01(const T *__restrict__ x,
                                                      T *__restrict__ out, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n)
        return;
    const T xx = x[i];
    T y;
    if (!special_value<T, KIND>(T(V), xx, &y)) {
        // binary32 order 1: between x3 and x1 the regime takes the Debye
        // branch (x3 < x1 there), so the scalar-order path does too and gives
        // the array path's bits
        constexpr RegimeSet r = Regime<T, KIND>::r;
        if constexpr (V == 1 && r.x3 < r.x1 && 1.0 > r.v3) {
            if (xx > T(r.x3) && !(xx > T(r.x1)))
                y = br_u<T, KIND>(T(V), xx);
            else
                y = order01<T, KIND, V>(xx);
        } else {
            y = order01<T, KIND, V>(xx);
        }
    }
    out[i] = y;
}

// Integer orders 2..14: one element per thread (order_int).
template <typename T, int KIND>
__global__ __launch_bounds__(kThreads) void k_order_int(int nu, const T *__restrict__ x,
                                                        T *__restrict__ out, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n)
        return;
    const T xx = x[i];
    T y;
    if (!special_value<T, KIND>(T(nu), xx, &y))
        y = order_int<T, KIND>(nu, xx);
    out[i] = y;
}

// ---------------------------------------------------------------------------
// Diagnostics kernels
// ---------------------------------------------------------------------------
template <typename T, int KIND>
__global__ __launch_bounds__(kThreads) void k_classify(const T *v, const T *x, uint8_t *br,
                                                       int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n)
        return;
    const T vv = (KIND == KIND_K) ? fabs(v[i]) : v[i];
    T y;
    br[i] = special_value<T, KIND>(vv, x[i], &y) ? uint8_t(BR_NONE)
                                                 : uint8_t(classify<T, KIND>(vv, x[i]));
}

// Integrand evaluations of the K fallback per element: the node count of the
// cosh-integral rule; 0 for every other branch, special value or sub-case
// (integer orders, x < 1e-10 and the Temme series at x <= 1.25 run no
// integral).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_knodes(const T *v, const T *x, int32_t *nodes,
                                                     int64_t n) {
    const auto *kt = ktab_for_kind<KIND_K, T>();
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n)
        return;
    const T vv = fabs(v[i]), xx = x[i];
    T y;
    int c = 0;
    // integer orders and x < 1e-10 take closed expansions, no integral
    if (!special_value<T, KIND_K>(vv, xx, &y) && classify<T, KIND_K>(vv, xx) == BR_FB &&
        xx >= T(1e-10) && !int_order(vv)) {
        if (xx <= T(tables::kTemmeX))
            c = 0;
        else if constexpr (std::is_same<T, float>::value)
            br_k_cosh32(vv, xx, kt, &c);
        else
            br_k_cosh(vv, xx, kt, &c);
    }
    nodes[i] = c;
}

// The library's binary64 elementary functions, one per element (op 0
// reciprocal, 1 exp, 2 exp of |a| < 1e9, 3 log, 4 log(1 + a)).
__global__ __launch_bounds__(kThreads) void k_elementary(int op, const double *a, double *out,
                                                         int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n)
        return;
    const double x = a[i];
    out[i] = (op == 0) ? lrcp(x) : (op == 1) ? lexp(x) : (op == 2) ? lexp_b(x)
             : (op == 3) ? llog(x) : (op == 4) ? llog1p(x) : lrsq(x);
}

// Series terms of the K fallback's Temme branch per element (after f_0); 0
// for every other branch, special value or sub-case.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_kterms(const T *v, const T *x, int32_t *terms,
                                                     int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n)
        return;
    const T vv = fabs(v[i]), xx = x[i];
    T y;
    int c = 0;
    if (!special_value<T, KIND_K>(vv, xx, &y) && classify<T, KIND_K>(vv, xx) == BR_FB &&
        xx >= T(1e-10) && xx <= T(tables::kTemmeX) && !int_order(vv))
        br_k_temme<T>(vv, xx, &c);
    terms[i] = c;
}

template <typename T, int KIND>
__global__ __launch_bounds__(kThreads) void k_branch(int b, const T *v, const T *x, T *out,
                                                     int64_t n) {
    const auto *kt = ktab_for_kind<KIND, T>();
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n)
        return;
    const T vv = (KIND == KIND_K) ? fabs(v[i]) : v[i];
    T y;
    if (!special_value<T, KIND>(vv, x[i], &y))
        y = eval_branch<T, KIND>(b, vv, x[i], kt);
    out[i] = y;
}

// ---------------------------------------------------------------------------
// von Mises-Fisher mean resultant: column sums of L2-normalised rows
// ---------------------------------------------------------------------------

// inv[i] = 1 / ||X[i, :]||_2 (0 for a zero row); one workgroup per row, sum of
// squares in binary64, fixed reduction order.
__global__ __launch_bounds__(kThreads) void k_rownorm_inv(const float *__restrict__ X, int64_t p,
                                                          double *__restrict__ inv) {
    const int64_t row = blockIdx.x;
    const float *r = X + row * p;
    double ss = 0.0;
    if ((p & 3) == 0 && (reinterpret_cast<uintptr_t>(r) & 15) == 0) {
        // 16-byte loads (same per-thread order: element 4j, 4j+1, ... of each load)
        const float4 *r4 = reinterpret_cast<const float4 *>(r);
        for (int64_t j = threadIdx.x; j < (p >> 2); j += kThreads) {
            const float4 a = r4[j];
            ss = fma(double(a.x), double(a.x), ss);
            ss = fma(double(a.y), double(a.y), ss);
            ss = fma(double(a.z), double(a.z), ss);
            ss = fma(double(a.w), double(a.w), ss);
        }
    } else {
        for (int64_t j = threadIdx.x; j < p; j += kThreads) {
            const double a = r[j];
            ss = fma(a, a, ss);
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        ss += __shfl_down(ss, off);
    __shared__ double part[kWaves];
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = (part[0] + part[1]) + (part[2] + part[3]);
        inv[row] = (t > 0.0) ? 1.0 / sqrt(t) : 0.0;
    }
}

// part[r, j] = sum over rows i of slice r of X[i, j] * inv[i] (binary64).
__global__ __launch_bounds__(kThreads) void k_colsum_part(const float *__restrict__ X,
                                                          const double *__restrict__ inv,
                                                          int64_t n, int64_t p, int64_t rows_per,
                                                          double *__restrict__ part) {
    const int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (j >= p)
        return;
    const int64_t r0 = int64_t(blockIdx.y) * rows_per;
    const int64_t r1 = (r0 + rows_per < n) ? r0 + rows_per : n;
    double s = 0.0;
    for (int64_t i = r0; i < r1; ++i)
        s = fma(double(X[i * p + j]), inv[i], s);
    part[int64_t(blockIdx.y) * p + j] = s;
}

// The same with four consecutive columns per thread and 16-byte loads (p a
// multiple of 4, X 16-byte aligned), four rows in flight per step; every
// column is still summed over its rows in order.
__global__ __launch_bounds__(kThreads) void k_colsum_part4(const float *__restrict__ X,
                                                           const double *__restrict__ inv,
                                                           int64_t n, int64_t p, int64_t rows_per,
                                                           double *__restrict__ part) {
    const int64_t j = (int64_t(blockIdx.x) * kThreads + threadIdx.x) * 4;
    if (j >= p)
        return;
    const int64_t r0 = int64_t(blockIdx.y) * rows_per;
    const int64_t r1 = (r0 + rows_per < n) ? r0 + rows_per : n;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t i = r0;
    for (; i + 4 <= r1; i += 4) {
        float4 a[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            a[k] = *reinterpret_cast<const float4 *>(X + (i + k) * p + j);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double w = inv[i + k];
            s0 = fma(double(a[k].x), w, s0);
            s1 = fma(double(a[k].y), w, s1);
            s2 = fma(double(a[k].z), w, s2);
            s3 = fma(double(a[k].w), w, s3);
        }
    }
    for (; i < r1; ++i) {
        const float4 a = *reinterpret_cast<const float4 *>(X + i * p + j);
        const double w = inv[i];
        s0 = fma(double(a.x), w, s0);
        s1 = fma(double(a.y), w, s1);
        s2 = fma(double(a.z), w, s2);
        s3 = fma(double(a.w), w, s3);
    }
    double *o = part + int64_t(blockIdx.y) * p + j;
    o[0] = s0;
    o[1] = s1;
    o[2] = s2;
    o[3] = s3;
}

// colsum[j] = sum_r part[r, j] in slice order.
__global__ __launch_bounds__(kThreads) void k_colsum_final(const double *__restrict__ part,
                                                           int64_t nslices, int64_t p,
                                                           double *__restrict__ colsum) {
    const int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (j >= p)
        return;
    double s = 0.0;
    for (int64_t r = 0; r < nslices; ++r)
        s += part[r * p + j];
    colsum[j] = s;
}

// *out = sum_j colsum[j]^2, one workgroup, fixed order.
__global__ __launch_bounds__(kThreads) void k_sumsq(const double *__restrict__ c, int64_t p,
                                                    double *__restrict__ out) {
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < p; j += kThreads)
        s = fma(c[j], c[j], s);
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_down(s, off);
    __shared__ double part[kWaves];
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        *out = (part[0] + part[1]) + (part[2] + part[3]);
}

// Maximum-likelihood kappa of a vMF fit from the column-sum pass (paper,
// eq. kappa estimates): R = sqrt(sumsq) / n, kappa_0 = R (p - R^2)/(1 - R^2),
// then kappa <- F(kappa) with A_p = exp(log I_{p/2} - log I_{p/2-1}) from the
// same branch code as the forward path, until the step is below 1e-15
// relative or no longer shrinks (the noise floor of A_p, whose two log-values
// are of size ~kappa), at most 40 steps.  One lane; out = {kappa, R, kappa_0,
// steps}.  The I series needs the log Gamma(1 + v) table in LDS (orders
// v <= 15, i.e. p <= 32, with kappa in the series region): every thread of
// the workgroup loads it before lane 0 solves.
__global__ __launch_bounds__(64) void k_vmf_kappa(const double *__restrict__ sumsq, int64_t n,
                                                  double p, double *__restrict__ out) {
    __shared__ LgTab lt;
    lgtab_load(&lt);
    if (threadIdx.x != 0)
        return;
    const double R = sqrt(*sumsq) / double(n);
    const double v = 0.5 * p - 1.0;
    double k = R * (p - R * R) / (1.0 - R * R);
    const double k0 = k;
    int it = 0;
    double prev = __builtin_inf();
    bool ok = (R > 0.0) && (R < 1.0) && (n > 0);
    for (; ok && it < 40; ++it) {
        const double l0 = eval_full<double, KIND_I>(v, k, &lt);
        const double l1 = eval_full<double, KIND_I>(v + 1.0, k, &lt);
        const double A = exp(l1 - l0);
        const double kn = k - (A - R) / (1.0 - A * A - (p - 1.0) * A / k);
        const double d = fabs(kn - k);
        const bool stop = (d <= 1e-15 * fabs(kn)) || (d >= prev);
        prev = d;
        k = kn;
        if (stop) {
            ++it;
            break;
        }
    }
    out[0] = ok ? k : __builtin_nan("");
    out[1] = R;
    out[2] = k0;
    out[3] = double(it);
}

}  // namespace lbessel

// ===========================================================================
// C-ABI
// ===========================================================================
using namespace lbessel;

namespace {

inline int launch_status() {
    return (hipGetLastError() == hipSuccess) ? LBESSEL_OK : LBESSEL_EHIP;
}

// Workspace of lbessel_vmf_fit_f32_noalloc: one copy per GPU, at its own
// address on each.  In host code the name stands for no device address: host
// code uses only the per-device pointer that hipGetSymbolAddress returns.
static __device__ __align__(256) double scratch[LBESSEL_VMF_FIT_STATIC_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of scratch per device id

// Device address of scratch on the current device, resolved on the first
// call per device and cached.
int static_scratch_on_current_device(void **ptr) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return LBESSEL_ENODEV;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return LBESSEL_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return LBESSEL_OK;
}

inline bool grid_ok(int64_t n, int per_block, uint32_t *blocks) {
    const int64_t b = (n + per_block - 1) / per_block;
    if (b > int64_t(0x7fffffff))
        return false;
    *blocks = uint32_t(b);
    return true;
}

template <typename T, int KIND, int OP>
int run_grouped(const T *v, const T *x, const T *g, T *out, int64_t n, T vs, T p, void *s) {
    if (n < 0)
        return LBESSEL_EINVAL;
    if (x == nullptr || out == nullptr || (!OpTraits<OP>::scalar_order && v == nullptr) ||
        (OP == OP_GRAD && g == nullptr)) {
        if (n > 0)
            return LBESSEL_EINVAL;
    }
    if (n == 0)
        return LBESSEL_OK;
    Args<T> a{v, x, g, out, n, vs, p};
    return launch_grouped<T, KIND, OP>(a, static_cast<hipStream_t>(s));
}

template <typename T, int KIND>
int run_ungrouped(const T *v, const T *x, T *out, int64_t n, void *s) {
    if (n < 0 || (n > 0 && (v == nullptr || x == nullptr || out == nullptr)))
        return LBESSEL_EINVAL;
    if (n == 0)
        return LBESSEL_OK;
    uint32_t blocks;
    if (!grid_ok(n, kThreads, &blocks))
        return LBESSEL_EINVAL;
    Args<T> a{v, x, nullptr, out, n, T(0), T(0)};
    hipLaunchKernelGGL((k_ungrouped<T, KIND, OP_LOG>), dim3(blocks), dim3(kThreads), 0,
                       static_cast<hipStream_t>(s), a);
    return launch_status();
}

template <typename T>
bool valid_dim(T p) {
    return p == p && p >= T(2) && p < T(__builtin_huge_val());
}

}  // namespace

extern "C" {

int lbessel_log_iv_f64(const double *v, const double *x, double *out, int64_t n, void *s) {
    return run_grouped<double, KIND_I, OP_LOG>(v, x, nullptr, out, n, 0.0, 0.0, s);
}
int lbessel_log_iv_f32(const float *v, const float *x, float *out, int64_t n, void *s) {
    return run_grouped<float, KIND_I, OP_LOG>(v, x, nullptr, out, n, 0.f, 0.f, s);
}
int lbessel_log_kv_f64(const double *v, const double *x, double *out, int64_t n, void *s) {
    return run_grouped<double, KIND_K, OP_LOG>(v, x, nullptr, out, n, 0.0, 0.0, s);
}
int lbessel_log_kv_f32(const float *v, const float *x, float *out, int64_t n, void *s) {
    return run_grouped<float, KIND_K, OP_LOG>(v, x, nullptr, out, n, 0.f, 0.f, s);
}

int lbessel_log_kv_integral_f64(const double *v, const double *x, double *out, int64_t n,
                                void *s) {
    if (n < 0 || (n > 0 && (v == nullptr || x == nullptr || out == nullptr)))
        return LBESSEL_EINVAL;
    if (n == 0)
        return LBESSEL_OK;
    Args<double> a{v, x, nullptr, out, n, 0.0, 0.0};
    return launch_grouped<double, KIND_K, OP_LOG, VAR_U_INTEGRAL>(a, static_cast<hipStream_t>(s));
}

int lbessel_log_iv_grad_x_f64(const double *v, const double *x, const double *g, double *gx,
                              int64_t n, void *s) {
    return run_grouped<double, KIND_I, OP_GRAD>(v, x, g, gx, n, 0.0, 0.0, s);
}
int lbessel_log_iv_grad_x_f32(const float *v, const float *x, const float *g, float *gx,
                              int64_t n, void *s) {
    return run_grouped<float, KIND_I, OP_GRAD>(v, x, g, gx, n, 0.f, 0.f, s);
}
int lbessel_log_kv_grad_x_f64(const double *v, const double *x, const double *g, double *gx,
                              int64_t n, void *s) {
    return run_grouped<double, KIND_K, OP_GRAD>(v, x, g, gx, n, 0.0, 0.0, s);
}
int lbessel_log_kv_grad_x_f32(const float *v, const float *x, const float *g, float *gx,
                              int64_t n, void *s) {
    return run_grouped<float, KIND_K, OP_GRAD>(v, x, g, gx, n, 0.f, 0.f, s);
}

int lbessel_vmf_log_norm_f64(const double *kappa, double p, double *out, int64_t n, void *s) {
    if (!valid_dim(p))
        return LBESSEL_EINVAL;
    return run_grouped<double, KIND_I, OP_VMF>(nullptr, kappa, nullptr, out, n, 0.5 * p - 1.0, p,
                                               s);
}
int lbessel_vmf_log_norm_f32(const float *kappa, float p, float *out, int64_t n, void *s) {
    if (!valid_dim(p))
        return LBESSEL_EINVAL;
    return run_grouped<float, KIND_I, OP_VMF>(nullptr, kappa, nullptr, out, n, 0.5f * p - 1.0f,
                                              p, s);
}
int lbessel_vmf_log_norm_grad_f64(const double *kappa, double p, double *out, int64_t n,
                                  void *s) {
    if (!valid_dim(p))
        return LBESSEL_EINVAL;
    return run_grouped<double, KIND_I, OP_VMF_GRAD>(nullptr, kappa, nullptr, out, n,
                                                    0.5 * p - 1.0, p, s);
}

}  // extern "C"

// Scalar order: orders 0 and 1 take the polynomial kernel (binary32 order 1
// between the Debye and Hankel bounds of x: the Debye branch), integer orders
// 2..14 of I the integer-order kernel, every other order the grouped kernel
// with the order broadcast (for K's integer orders its fallback runs the
// same integer-order code, and the grouping keeps the recurrence and the
// Hankel elements in separate chunks: 0.31 -> 0.20 ms for 20M x in [0, 150)).
template <typename T, int KIND>
static int run_order(T v, const T *x, T *out, int64_t n, hipStream_t st) {
    if (n < 0)
        return LBESSEL_EINVAL;
    if (n == 0)
        return LBESSEL_OK;
    if (x == nullptr || out == nullptr)
        return LBESSEL_EINVAL;
    const T av = (KIND == KIND_K) ? fabs(v) : v;
    uint32_t blocks;
    if (av == T(0) || av == T(1)) {
        if (!grid_ok(n, kThreads, &blocks))
            return LBESSEL_EINVAL;
        if (av == T(0))
            hipLaunchKernelGGL((k_order01<T, KIND, 0>), dim3(blocks), dim3(kThreads), 0, st, x,
                               out, n);
        else
            hipLaunchKernelGGL((k_order01<T, KIND, 1>), dim3(blocks), dim3(kThreads), 0, st, x,
                               out, n);
        return launch_status();
    }
    if constexpr (KIND == KIND_I) {
        if (av == rint(av) && av >= T(tables::kIntOrderMin) && av <= T(tables::kIntOrderMax)) {
            if (!grid_ok(n, kThreads, &blocks))
                return LBESSEL_EINVAL;
            hipLaunchKernelGGL((k_order_int<T, KIND>), dim3(blocks), dim3(kThreads), 0, st,
                               int(av), x, out, n);
            return launch_status();
        }
    }
    Args<T> a{nullptr, x, nullptr, out, n, v, T(0)};
    return launch_grouped<T, KIND, OP_LOG>(a, st);
}

extern "C" {

int lbessel_log_iv_order_f64(double v, const double *x, double *out, int64_t n, void *s) {
    return run_order<double, KIND_I>(v, x, out, n, static_cast<hipStream_t>(s));
}
int lbessel_log_kv_order_f64(double v, const double *x, double *out, int64_t n, void *s) {
    return run_order<double, KIND_K>(v, x, out, n, static_cast<hipStream_t>(s));
}
int lbessel_log_iv_order_f32(float v, const float *x, float *out, int64_t n, void *s) {
    return run_order<float, KIND_I>(v, x, out, n, static_cast<hipStream_t>(s));
}
int lbessel_log_kv_order_f32(float v, const float *x, float *out, int64_t n, void *s) {
    return run_order<float, KIND_K>(v, x, out, n, static_cast<hipStream_t>(s));
}

int lbessel_k_nodes(int precision, const void *v, const void *x, int32_t *nodes, int64_t n,
                    void *s) {
    if (n < 0 || (precision != 64 && precision != 32))
        return LBESSEL_EINVAL;
    if (n == 0)
        return LBESSEL_OK;
    if (v == nullptr || x == nullptr || nodes == nullptr)
        return LBESSEL_EINVAL;
    uint32_t blocks;
    if (!grid_ok(n, kThreads, &blocks))
        return LBESSEL_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(s);
    if (precision == 64)
        hipLaunchKernelGGL(k_knodes<double>, dim3(blocks), dim3(kThreads), 0, st,
                           (const double *)v, (const double *)x, nodes, n);
    else
        hipLaunchKernelGGL(k_knodes<float>, dim3(blocks), dim3(kThreads), 0, st,
                           (const float *)v, (const float *)x, nodes, n);
    return launch_status();
}

int lbessel_elementary_f64(int op, const double *a, double *out, int64_t n, void *s) {
    if (n < 0 || op < 0 || op > 5)
        return LBESSEL_EINVAL;
    if (n == 0)
        return LBESSEL_OK;
    if (a == nullptr || out == nullptr)
        return LBESSEL_EINVAL;
    uint32_t blocks;
    if (!grid_ok(n, kThreads, &blocks))
        return LBESSEL_EINVAL;
    hipLaunchKernelGGL(k_elementary, dim3(blocks), dim3(kThreads), 0, static_cast<hipStream_t>(s),
                       op, a, out, n);
    return launch_status();
}

int lbessel_k_terms(int precision, const void *v, const void *x, int32_t *terms, int64_t n,
                    void *s) {
    if (n < 0 || (precision != 64 && precision != 32))
        return LBESSEL_EINVAL;
    if (n == 0)
        return LBESSEL_OK;
    if (v == nullptr || x == nullptr || terms == nullptr)
        return LBESSEL_EINVAL;
    uint32_t blocks;
    if (!grid_ok(n, kThreads, &blocks))
        return LBESSEL_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(s);
    if (precision == 64)
        hipLaunchKernelGGL(k_kterms<double>, dim3(blocks), dim3(kThreads), 0, st,
                           (const double *)v, (const double *)x, terms, n);
    else
        hipLaunchKernelGGL(k_kterms<float>, dim3(blocks), dim3(kThreads), 0, st,
                           (const float *)v, (const float *)x, terms, n);
    return launch_status();
}

int lbessel_classify(int kind, int precision, const void *v, const void *x, uint8_t *branch,
                     int64_t n, void *s) {
    if (n < 0 || (kind != 0 && kind != 1) || (precision != 64 && precision != 32))
        return LBESSEL_EINVAL;
    if (n == 0)
        return LBESSEL_OK;
    if (v == nullptr || x == nullptr || branch == nullptr)
        return LBESSEL_EINVAL;
    uint32_t blocks;
    if (!grid_ok(n, kThreads, &blocks))
        return LBESSEL_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(s);
    if (precision == 64) {
        if (kind == 0)
            hipLaunchKernelGGL((k_classify<double, KIND_I>), dim3(blocks), dim3(kThreads), 0, st,
                               (const double *)v, (const double *)x, branch, n);
        else
            hipLaunchKernelGGL((k_classify<double, KIND_K>), dim3(blocks), dim3(kThreads), 0, st,
                               (const double *)v, (const double *)x, branch, n);
    } else {
        if (kind == 0)
            hipLaunchKernelGGL((k_classify<float, KIND_I>), dim3(blocks), dim3(kThreads), 0, st,
                               (const float *)v, (const float *)x, branch, n);
        else
            hipLaunchKernelGGL((k_classify<float, KIND_K>), dim3(blocks), dim3(kThreads), 0, st,
                               (const float *)v, (const float *)x, branch, n);
    }
    return launch_status();
}

}  // extern "C"

template <typename T>
static int run_branch(int kind, int branch, const T *v, const T *x, T *out, int64_t n,
                      void *s) {
    if (n < 0 || (kind != 0 && kind != 1) || branch < 0 || branch > 2)
        return LBESSEL_EINVAL;
    if (n == 0)
        return LBESSEL_OK;
    if (v == nullptr || x == nullptr || out == nullptr)
        return LBESSEL_EINVAL;
    uint32_t blocks;
    if (!grid_ok(n, kThreads, &blocks))
        return LBESSEL_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(s);
    if (kind == 0)
        hipLaunchKernelGGL((k_branch<T, KIND_I>), dim3(blocks), dim3(kThreads), 0, st, branch, v,
                           x, out, n);
    else
        hipLaunchKernelGGL((k_branch<T, KIND_K>), dim3(blocks), dim3(kThreads), 0, st, branch, v,
                           x, out, n);
    return launch_status();
}

extern "C" {

int lbessel_eval_branch_f64(int kind, int branch, const double *v, const double *x, double *out,
                            int64_t n, void *s) {
    return run_branch<double>(kind, branch, v, x, out, n, s);
}

int lbessel_eval_branch_f32(int kind, int branch, const float *v, const float *x, float *out,
                            int64_t n, void *s) {
    return run_branch<float>(kind, branch, v, x, out, n, s);
}

int lbessel_eval_ungrouped(int kind, int precision, const void *v, const void *x, void *out,
                           int64_t n, void *s) {
    if ((kind != 0 && kind != 1) || (precision != 64 && precision != 32))
        return LBESSEL_EINVAL;
    if (precision == 64) {
        if (kind == 0)
            return run_ungrouped<double, KIND_I>((const double *)v, (const double *)x,
                                                 (double *)out, n, s);
        return run_ungrouped<double, KIND_K>((const double *)v, (const double *)x, (double *)out,
                                             n, s);
    }
    if (kind == 0)
        return run_ungrouped<float, KIND_I>((const float *)v, (const float *)x, (float *)out, n,
                                            s);
    return run_ungrouped<float, KIND_K>((const float *)v, (const float *)x, (float *)out, n, s);
}

// Row slices of the column-sum pass: enough workgroups to fill the chip
// (>= 2048) while every slice keeps >= 64 rows.
// Columns per thread of the column-sum pass: 4 with 16-byte loads for wide
// rows (p >= 4096) that start 16-byte aligned, else 1.  Narrower rows keep
// one column per thread: four would leave too few column blocks, and the
// extra slices cost more in the final reduction than the wider loads save.
static int vmf_cols_per_thread(const void *X, int64_t p) {
    return (p >= 4096 && (p & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0) ? 4 : 1;
}

static int64_t vmf_slices(int64_t n, int64_t p, int cpt) {
    const int64_t col_blocks = (p + int64_t(kThreads) * cpt - 1) / (int64_t(kThreads) * cpt);
    int64_t r = (2048 + col_blocks - 1) / col_blocks;
    const int64_t max_r = (n + 63) / 64;
    if (r > max_r)
        r = max_r;
    if (r < 1)
        r = 1;
    if (r > 65535)
        r = 65535;
    return r;
}

int64_t lbessel_vmf_colsum_workspace(int64_t n, int64_t p) {
    if (n < 0 || p < 0)
        return LBESSEL_EINVAL;
    // the 4-column pass (when taken) uses the most slices; the 1-column pass
    // fits inside
    const int cpt = (p >= 4096 && (p & 3) == 0) ? 4 : 1;
    return (vmf_slices(n, p, cpt) * p + n) * int64_t(sizeof(double));
}

int lbessel_vmf_colsum_f32(const float *X, int64_t n, int64_t p, double *colsum, double *sumsq,
                           void *work, int64_t work_bytes, void *s) {
    if (n < 0 || p < 0 || n > int64_t(0x7fffffff))
        return LBESSEL_EINVAL;
    if (p == 0)
        return LBESSEL_OK;
    const int64_t need = lbessel_vmf_colsum_workspace(n, p);
    if (colsum == nullptr || work == nullptr || work_bytes < need || (n > 0 && X == nullptr))
        return LBESSEL_EINVAL;
    const int cpt = vmf_cols_per_thread(X, p);
    const int64_t slices = vmf_slices(n, p, cpt);
    const int64_t rows_per = (n + slices - 1) / slices;
    const int64_t col_blocks = (p + kThreads - 1) / kThreads;
    const int64_t col_blocks_cpt = (p + int64_t(kThreads) * cpt - 1) / (int64_t(kThreads) * cpt);
    if (col_blocks > int64_t(0x7fffffff))
        return LBESSEL_EINVAL;
    double *part = static_cast<double *>(work);
    double *inv = part + slices * p;
    hipStream_t st = static_cast<hipStream_t>(s);
    if (n > 0)
        hipLaunchKernelGGL(k_rownorm_inv, dim3(uint32_t(n)), dim3(kThreads), 0, st, X, p, inv);
    if (cpt == 4)
        hipLaunchKernelGGL(k_colsum_part4, dim3(uint32_t(col_blocks_cpt), uint32_t(slices)),
                           dim3(kThreads), 0, st, X, inv, n, p, rows_per, part);
    else
        hipLaunchKernelGGL(k_colsum_part, dim3(uint32_t(col_blocks), uint32_t(slices)),
                           dim3(kThreads), 0, st, X, inv, n, p, rows_per, part);
    hipLaunchKernelGGL(k_colsum_final, dim3(uint32_t(col_blocks)), dim3(kThreads), 0, st, part,
                       slices, p, colsum);
    if (sumsq != nullptr)
        hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(kThreads), 0, st, colsum, p, sumsq);
    return launch_status();
}

int lbessel_vmf_fit_f32(const float *X, int64_t n, int64_t p, double *result, void *work,
                        int64_t work_bytes, void *s) {
    if (n < 1 || p < 2 || result == nullptr)
        return LBESSEL_EINVAL;
    const int64_t need = lbessel_vmf_colsum_workspace(n, p);
    if (work == nullptr || work_bytes < need + int64_t((p + 1) * sizeof(double)))
        return LBESSEL_EINVAL;
    double *colsum = reinterpret_cast<double *>(static_cast<char *>(work) + need);
    double *sumsq = colsum + p;
    const int rc = lbessel_vmf_colsum_f32(X, n, p, colsum, sumsq, work, need, s);
    if (rc != LBESSEL_OK)
        return rc;
    hipLaunchKernelGGL(k_vmf_kappa, dim3(1), dim3(64), 0, static_cast<hipStream_t>(s), sumsq, n,
                       double(p), result);
    return launch_status();
}

int64_t lbessel_vmf_fit_workspace(int64_t n, int64_t p) {
    const int64_t w = lbessel_vmf_colsum_workspace(n, p);
    return (w < 0) ? w : w + (p + 1) * int64_t(sizeof(double));
}

int lbessel_vmf_fit_f32_noalloc(const float *X, int64_t n, int64_t p, double *result, void *s) {
    constexpr int64_t cap = LBESSEL_VMF_FIT_STATIC_BYTES;
    if (n < 1 || p < 2 || X == nullptr || result == nullptr)
        return LBESSEL_EINVAL;
    // the workspace holds at least p + n doubles: bound both before sizing it
    if (p > cap / int64_t(sizeof(double)) || n > cap / int64_t(sizeof(double)))
        return LBESSEL_ENOSPACE;
    const int64_t need = lbessel_vmf_fit_workspace(n, p);
    if (need < 0)
        return LBESSEL_EINVAL;
    if (need > cap)
        return LBESSEL_ENOSPACE;
    void *work = nullptr;
    const int rc = static_scratch_on_current_device(&work);
    if (rc != LBESSEL_OK)
        return rc;
    return lbessel_vmf_fit_f32(X, n, p, result, work, cap, s);
}

int lbessel_eval_segments(int kind, int precision, const lbessel_segment_t *segs, int nseg,
                          int64_t tiles, void *s) {
    if ((kind != 0 && kind != 1) || (precision != 64 && precision != 32) || nseg < 0 ||
        tiles < 0 || tiles > int64_t(0x7fffffff))
        return LBESSEL_EINVAL;
    if (nseg == 0 || tiles == 0)
        return LBESSEL_OK;
    if (segs == nullptr)
        return LBESSEL_EINVAL;
    const lbessel_segment_t *sg = segs;
    hipStream_t st = static_cast<hipStream_t>(s);
    const dim3 grid{uint32_t(tiles)}, block{kThreads};
    if (precision == 64) {
        if (kind == 0)
            hipLaunchKernelGGL((k_grouped_seg<double, KIND_I>), grid, block, 0, st, sg, nseg);
        else
            hipLaunchKernelGGL((k_grouped_seg<double, KIND_K>), grid, block, 0, st, sg, nseg);
    } else {
        if (kind == 0)
            hipLaunchKernelGGL((k_grouped_seg<float, KIND_I>), grid, block, 0, st, sg, nseg);
        else
            hipLaunchKernelGGL((k_grouped_seg<float, KIND_K>), grid, block, 0, st, sg, nseg);
    }
    return launch_status();
}

int lbessel_eval_segments_inline(int kind, int precision, const lbessel_segment_t *segs,
                                 int nseg, int64_t tiles, void *s) {
    if ((kind != 0 && kind != 1) || (precision != 64 && precision != 32) || nseg < 0 ||
        nseg > LBESSEL_SEG_INLINE_MAX || tiles < 0 || tiles > int64_t(0x7fffffff))
        return LBESSEL_EINVAL;
    if (nseg == 0 || tiles == 0)
        return LBESSEL_OK;
    if (segs == nullptr)
        return LBESSEL_EINVAL;
    SegPack pack{};
    for (int k = 0; k < nseg; ++k)
        pack.s[k] = segs[k];
    hipStream_t st = static_cast<hipStream_t>(s);
    const dim3 grid{uint32_t(tiles)}, block{kThreads};
    if (precision == 64) {
        if (kind == 0)
            hipLaunchKernelGGL((k_grouped_seg_inline<double, KIND_I>), grid, block, 0, st, pack,
                               nseg);
        else
            hipLaunchKernelGGL((k_grouped_seg_inline<double, KIND_K>), grid, block, 0, st, pack,
                               nseg);
    } else {
        if (kind == 0)
            hipLaunchKernelGGL((k_grouped_seg_inline<float, KIND_I>), grid, block, 0, st, pack,
                               nseg);
        else
            hipLaunchKernelGGL((k_grouped_seg_inline<float, KIND_K>), grid, block, 0, st, pack,
                               nseg);
    }
    return launch_status();
}

int64_t lbessel_segment_tiles(int64_t n) {
    if (n < 0)
        return LBESSEL_EINVAL;
    return (n + TileCfg<1>::tile - 1) / TileCfg<1>::tile;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Variants and layouts (measurement)
// ---------------------------------------------------------------------------
static int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

static size_t sort_temp_bytes(int64_t n) {
    size_t temp = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, temp, static_cast<const uint8_t *>(nullptr),
                                       static_cast<uint8_t *>(nullptr),
                                       static_cast<const uint32_t *>(nullptr),
                                       static_cast<uint32_t *>(nullptr), int(n), 0, 3);
    return temp;
}

extern "C" int64_t lbessel_eval_variant_workspace(int64_t n) {
    if (n < 0 || n > int64_t(0x7fffffff))
        return LBESSEL_EINVAL;
    if (n == 0)
        return 0;
    return 2 * align256(n) + 2 * align256(4 * n) + align256(int64_t(sort_temp_bytes(n)));
}

template <int KIND, int VAR>
static int run_variant(int layout, const double *v, const double *x, double *out, int64_t n,
                       void *work, int64_t work_bytes, hipStream_t st) {
    Args<double> a{v, x, nullptr, out, n, 0.0, 0.0};
    uint32_t blocks;
    if (layout == LBESSEL_LAYOUT_GROUPED) {
        if (VAR == VAR_SEVEN)
            return LBESSEL_EINVAL;
        return launch_grouped<double, KIND, OP_LOG, (VAR == VAR_SEVEN ? 0 : VAR)>(a, st);
    }
    if (!grid_ok(n, kThreads, &blocks))
        return LBESSEL_EINVAL;
    if (layout == LBESSEL_LAYOUT_NAIVE) {
        hipLaunchKernelGGL((k_ungrouped<double, KIND, OP_LOG, VAR>), dim3(blocks), dim3(kThreads),
                           0, st, a);
        return launch_status();
    }
    // LBESSEL_LAYOUT_SORTED
    const int64_t need = lbessel_eval_variant_workspace(n);
    if (need < 0 || work == nullptr || work_bytes < need)
        return LBESSEL_EINVAL;
    char *w = static_cast<char *>(work);
    uint8_t *k0 = reinterpret_cast<uint8_t *>(w);
    uint8_t *k1 = reinterpret_cast<uint8_t *>(w + align256(n));
    uint32_t *i0 = reinterpret_cast<uint32_t *>(w + 2 * align256(n));
    uint32_t *i1 = reinterpret_cast<uint32_t *>(w + 2 * align256(n) + align256(4 * n));
    void *temp = w + 2 * align256(n) + 2 * align256(4 * n);
    size_t temp_bytes = sort_temp_bytes(n);
    hipLaunchKernelGGL((k_sort_keys<KIND, VAR>), dim3(blocks), dim3(kThreads), 0, st, v, x, k0,
                       i0, n);
    if (hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, k0, k1, i0, i1, int(n), 0, 3, st) !=
        hipSuccess)
        return LBESSEL_EHIP;
    hipLaunchKernelGGL((k_sorted_eval<KIND, VAR>), dim3(blocks), dim3(kThreads), 0, st, k1, i1,
                       v, x, out, n);
    return launch_status();
}

template <int KIND>
static int run_variant_kind(int variant, int layout, const double *v, const double *x,
                            double *out, int64_t n, void *work, int64_t work_bytes,
                            hipStream_t st) {
    switch (variant) {
    case VAR_DEFAULT: return run_variant<KIND, VAR_DEFAULT>(layout, v, x, out, n, work, work_bytes, st);
    case VAR_PAPER_REGIMES: return run_variant<KIND, VAR_PAPER_REGIMES>(layout, v, x, out, n, work, work_bytes, st);
    case VAR_U_INTEGRAL: return run_variant<KIND, VAR_U_INTEGRAL>(layout, v, x, out, n, work, work_bytes, st);
    case VAR_SIMPSON: return run_variant<KIND, VAR_SIMPSON>(layout, v, x, out, n, work, work_bytes, st);
    case VAR_PAPER: return run_variant<KIND, VAR_PAPER>(layout, v, x, out, n, work, work_bytes, st);
    case VAR_SEVEN: return run_variant<KIND, VAR_SEVEN>(layout, v, x, out, n, work, work_bytes, st);
    default: return LBESSEL_EINVAL;
    }
}

extern "C" {

int lbessel_eval_variant(int kind, int variant, int layout, const double *v, const double *x,
                         double *out, int64_t n, void *work, int64_t work_bytes, void *s) {
    if ((kind != 0 && kind != 1) || variant < 0 || variant >= VAR_COUNT || layout < 0 ||
        layout > LBESSEL_LAYOUT_SORTED || n < 0 || n > int64_t(0x7fffffff))
        return LBESSEL_EINVAL;
    if (layout == LBESSEL_LAYOUT_GROUPED && variant == VAR_SEVEN)
        return LBESSEL_EINVAL;
    if (n == 0)
        return LBESSEL_OK;
    if (v == nullptr || x == nullptr || out == nullptr)
        return LBESSEL_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(s);
    return (kind == 0) ? run_variant_kind<KIND_I>(variant, layout, v, x, out, n, work, work_bytes, st)
                       : run_variant_kind<KIND_K>(variant, layout, v, x, out, n, work, work_bytes, st);
}

int lbessel_abi_version(void) { return LBESSEL_ABI_VERSION; }

const char *lbessel_status_string(int status) {
    switch (status) {
    case LBESSEL_OK: return "ok";
    case LBESSEL_EINVAL: return "invalid argument";
    case LBESSEL_EHIP: return "HIP launch failure";
    case LBESSEL_ENODEV: return "no usable device";
    case LBESSEL_ENOSPACE: return "request larger than the static buffer";
    case LBESSEL_ETOOBIG: return "request larger than the server arena";
    case LBESSEL_ETIMEOUT: return "timed out";
    case LBESSEL_ESTOPPED: return "server stopped";
    default: return "unknown status";
    }
}

}  // extern "C"
