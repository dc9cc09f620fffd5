// Serving step kernels: one level-synchronous step advances every admitted
// request by one stage (paper Sec. II.C: levels in sequence; a step keeps each
// request's levels in order while different requests share the launch, the
// many configurations in flight of Sec. II.C and Sec. III).
//
// A step is a graph: the upload of the step table, then independent kernels
// that read it, one per section.  serve_fused_kernel (16 waves, levels in
// LDS) sweeps whole narrow graphs, 64 samples per item; serve_stream_kernel
// (4 waves, the shape of the standalone streamed kernels) runs one interior
// level, the final-node partial sums or the final combine of the wide graphs.
// Each is instantiated per edge-factor kind (rational, lookup), so that the
// rational kernels keep their own register budget.
// Work items are numbered per section and taken grid-stride.  Every item runs
// the same device routines as the standalone kernels, so a request's result is
// bit-identical to cos_evaluate alone, whatever it shares a step with.
#include <atomic>

#include "fused_plan.h"
#include "serve_types.h"
#include "sweep_device.h"

namespace cosdag {
namespace {

constexpr int kServeFusedGrid = 256;    // one 16-wave group per CU
constexpr int kServeStreamGrid = 2048;  // eight 4-wave groups per CU

// Entry of [lo, lo + n) whose items contain `item` (item_base ascending).
__device__ __forceinline__ uint32_t find_entry(const StepTable *__restrict__ t, uint32_t lo, uint32_t n,
                                               uint32_t item) {
    uint32_t hi = lo + n - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (t->e[mid].item_base <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename T, int RMAX, bool RESCALE, int KIND>
__device__ __forceinline__ void serve_fused(const ServeReqDev &r, uint32_t tile, unsigned char *lds, int wave,
                                            int lane) {
    if constexpr (acc_fits(sizeof(T), 1, RMAX)) {
        const FusedGraph G{r.row_ptr, r.edges, r.edges32, r.edgesL, r.levels, r.L, r.x, r.S, r.out, r.out_exp};
        fused_tile<T, 1, RMAX, RESCALE, KIND>(G, static_cast<int64_t>(tile) * kWave, reinterpret_cast<T *>(lds),
                                              reinterpret_cast<uint32_t *>(lds + r.off_red),
                                              reinterpret_cast<double *>(lds + r.off_part), wave, lane);
    }
}

template <typename T, bool RESCALE, int KIND>
__device__ __forceinline__ void serve_fused_rows(const ServeReqDev &r, uint32_t tile, unsigned char *lds, int wave,
                                                 int lane) {
    switch (r.rows_variant) {
    case 2:
        serve_fused<T, 2, RESCALE, KIND>(r, tile, lds, wave, lane);
        break;
    case 4:
        serve_fused<T, 4, RESCALE, KIND>(r, tile, lds, wave, lane);
        break;
    case 8:
        serve_fused<T, 8, RESCALE, KIND>(r, tile, lds, wave, lane);
        break;
    case 16:
        serve_fused<T, 16, RESCALE, KIND>(r, tile, lds, wave, lane);
        break;
    case 24:
        serve_fused<T, 24, RESCALE, KIND>(r, tile, lds, wave, lane);
        break;
    default:
        serve_fused<T, kMaxRows, RESCALE, KIND>(r, tile, lds, wave, lane);
        break;
    }
}

// Interior level l for a row group of 32 rows (8 per wave) and a tile of 256
// samples; the level buffers (values of type V) alternate as in the standalone
// sweep, and so do the exponent rows: level l is scaled by row l-1 (row 0 holds
// level 1's headroom, 0 unless binary16) and folds its largest |value|, times
// 2^h_{l+1} for binary16, into row l.
template <typename T, bool RESCALE, int KIND, typename V>
__device__ __forceinline__ void serve_level(const ServeReqDev &r, int l, uint32_t local, uint32_t n_rg,
                                            uint32_t *red, int wave, int lane) {
    constexpr int K = kServeLevelK;
    const uint32_t rg = local % n_rg;
    const uint32_t tile = local / n_rg;
    const int64_t tbase = static_cast<int64_t>(tile) * (kWave * K);
    const LevelDev lv = load_level(r.levels, l - 1);
    V *const b0 = reinterpret_cast<V *>(r.ws + r.off_buf0);
    V *const b1 = reinterpret_cast<V *>(r.ws + r.off_buf1);
    V *cur = (l - 1) & 1 ? b1 : b0;
    const V *prev = (l - 2) & 1 ? b1 : b0;
    uint32_t *maxbits = reinterpret_cast<uint32_t *>(r.ws + r.off_maxbits);
    typename SweepPath<T, KIND>::template Samples<K> smp;
    if constexpr (KIND == FK_LOOKUP_T32)
        smp.load(r.t32, r.S, r.S_pad, tbase, lane);
    else
        smp.load(r.x, r.S, r.S, tbase, lane);
    const typename SweepPath<T, KIND>::Rec *recs;
    if constexpr (KIND != FK_RATIONAL)
        recs = r.edgesL;
    else if constexpr (sizeof(T) == sizeof(double))
        recs = r.edges;
    else
        recs = r.edges32;
    int esh[K];
    uint32_t lmax[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        esh[m] = RESCALE ? ilogb_bits(maxbits[static_cast<int64_t>(l - 1) * r.S_pad + tbase + lane + kWave * m]) : 0;
        lmax[m] = 0u;
    }
    const int jbeg = min(static_cast<int>(rg) * kServeLevelRowsPerItem + wave * kServeLevelRows, lv.w_dst);
    const int jend = min(jbeg + kServeLevelRows, lv.w_dst);
    const int32_t *rp = r.row_ptr + lv.rp_begin;
    if (l == 1)
        level_wave_rows<T, K, true, RESCALE, KIND, V>(rp, recs, jbeg, jend, nullptr, cur, r.S_pad, tbase, lane, smp,
                                                      esh, lmax);
    else
        level_wave_rows<T, K, false, RESCALE, KIND, V>(rp, recs, jbeg, jend, prev, cur, r.S_pad, tbase, lane, smp,
                                                       esh, lmax);
    if constexpr (RESCALE) {
        if (l <= r.L - 2) {
            if constexpr (std::is_same_v<V, _Float16>) {
                const int32_t h_next = r.h16[l + 1];
                if (h_next)  // exact: |value| <= 2^15 and h_next <= 96
#pragma unroll
                    for (int m = 0; m < K; ++m)
                        lmax[m] = abs_bits(ldexpf(__uint_as_float(lmax[m]), h_next));
            }
            fold_max<K, 4>(red, lmax, wave, lane, maxbits + static_cast<int64_t>(l) * r.S_pad + tbase);
        }
    }
}

// Final-node partial sums of one chunk of 256 edges (wave w: quarter w) for a
// tile of 128 samples, combined as ((q0 + q1) + q2) + q3 exactly as
// final_partial_kernel does.
template <typename TV, int KIND>
__device__ __forceinline__ void serve_final(const ServeReqDev &r, uint32_t local, double *red, int wave, int lane) {
    constexpr int K = kServeFinalK;
    const uint32_t n_chunks = static_cast<uint32_t>(r.final_chunks);
    const int c = static_cast<int>(local % n_chunks);
    const int64_t tbase = static_cast<int64_t>(local / n_chunks) * (kWave * K);
    const LevelDev lf = load_level(r.levels, r.L - 1);
    typename FinalPath<KIND>::template Samples<K> smp;
    smp.load(r.x, r.S, r.S, tbase, lane);
    const int c_end = min((c + 1) * kFinalChunk, lf.n_edges);
    const int e_lo = min(c * kFinalChunk + wave * kQuarter, c_end);
    const int e_hi = min(e_lo + kQuarter, c_end);
    double acc[K];
    const typename FinalPath<KIND>::Rec *edges;
    if constexpr (KIND == FK_LOOKUP)
        edges = r.edgesL + lf.e_begin;
    else
        edges = r.edges + lf.e_begin;
    if (r.L == 1) {
        final_quarter<double, K, true, KIND>(edges, e_lo, e_hi, nullptr, r.S_pad, tbase, lane, smp, acc);
    } else {
        const TV *prev = reinterpret_cast<const TV *>(r.ws + ((r.L - 2) & 1 ? r.off_buf1 : r.off_buf0));
        final_quarter<TV, K, false, KIND>(edges, e_lo, e_hi, prev, r.S_pad, tbase, lane, smp, acc);
    }
#pragma unroll
    for (int m = 0; m < K; ++m)
        red[wave * (kWave * K) + lane + kWave * m] = acc[m];
    __syncthreads();
    double *partial = reinterpret_cast<double *>(r.ws + r.off_partial);
    for (int i = threadIdx.x; i < kWave * K; i += kBlock)
        partial[static_cast<int64_t>(c) * r.S_pad + tbase + i] =
            ((red[i] + red[kWave * K + i]) + red[2 * kWave * K + i]) + red[3 * kWave * K + i];
}

// Whole-graph items of section SEC (SS_FUSED, or SS_FUSED_LOOKUP with KIND lookup).
template <int KIND, uint32_t SEC>
__global__ __launch_bounds__(kFusedThreads) void serve_fused_kernel(const StepTable *__restrict__ tab,
                                                                    const ServeReqDev *__restrict__ reqs) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lo = section_begin(*tab, SEC);
    const uint32_t n = tab->n[SEC];
    const uint32_t total = tab->items[SEC];
    for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
        const StepEntry &en = tab->e[find_entry(tab, lo, n, item)];
        const ServeReqDev &r = reqs[en.slot];
        const uint32_t tile = item - en.item_base;
        if (r.precision == COS_FP64)
            serve_fused_rows<double, false, KIND>(r, tile, lds, wave, lane);
        else if (r.precision == COS_FP32_RESCALED)
            serve_fused_rows<float, true, KIND>(r, tile, lds, wave, lane);
        else
            serve_fused_rows<float, false, KIND>(r, tile, lds, wave, lane);
        // fused_tile ends with a group barrier, so LDS is free for the next item
    }
}

// Level, final-node and combine items of section SEC (SS_STREAMED, or
// SS_STREAMED_LOOKUP with KIND lookup, where the binary32 precisions read the
// binary32 copy of the tables made by the request's first stage).
template <int KIND, uint32_t SEC>
__global__ __launch_bounds__(kBlock) void serve_stream_kernel(StepTable *__restrict__ tab,
                                                              const ServeReqDev *__restrict__ reqs) {
    __shared__ __align__(16) unsigned char lds[4 * kWave * kServeLevelK * sizeof(uint32_t)];
    __shared__ uint32_t claim;
    static_assert(sizeof(lds) >= 4 * kWave * kServeFinalK * sizeof(double), "final-node staging");
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lo = section_begin(*tab, SEC);
    const uint32_t n = tab->n[SEC];
    const uint32_t total = tab->items[SEC];
    // items cost different amounts (they belong to different requests), so a
    // workgroup claims its next item when it is done with the last: items
    // c, c + 8, c + 16, ... from the counter of c = the workgroup's XCD (eight
    // counters, so that claims do not all serialise on one address)
    const uint32_t c = blockIdx.x % kXcds;
    for (;;) {
        if (threadIdx.x == 0)
            claim = c + kXcds * atomicAdd(&tab->claimed[SEC][c].v, 1u);
        __syncthreads();
        const uint32_t item = claim;
        if (item >= total)
            break;
        const StepEntry &en = tab->e[find_entry(tab, lo, n, item)];
        const ServeReqDev &r = reqs[en.slot];
        const uint32_t local = item - en.item_base;
        const uint32_t kind = en.kind;
        if (kind == SK_LEVEL) {
            constexpr int K32 = KIND == FK_LOOKUP ? FK_LOOKUP_T32 : KIND;  // kind of the binary32 levels
            const int l = static_cast<int>(en.level);
            uint32_t *red = reinterpret_cast<uint32_t *>(lds);
            if (r.precision == COS_FP64)
                serve_level<double, false, KIND, double>(r, l, local, en.n_rg, red, wave, lane);
            else if (r.precision == COS_FP32_RESCALED)
                serve_level<float, true, K32, float>(r, l, local, en.n_rg, red, wave, lane);
            else if (r.precision == COS_BF16_RESCALED)
                serve_level<float, true, K32, __bf16>(r, l, local, en.n_rg, red, wave, lane);
            else if (r.precision == COS_FP16_RESCALED) {
                if constexpr (KIND == FK_RATIONAL)  // binary16 needs the factors' bound: rational only
                    serve_level<float, true, KIND, _Float16>(r, l, local, en.n_rg, red, wave, lane);
            } else
                serve_level<float, false, K32, float>(r, l, local, en.n_rg, red, wave, lane);
        } else if (kind == SK_TABLE32) {
            // entries [local * 256, local * 256 + 256) of [n_slots][S_pad] (S_pad a multiple of 256)
            if constexpr (KIND == FK_LOOKUP) {
                const int64_t i = static_cast<int64_t>(local) * kServeCombineTile + threadIdx.x;
                const int64_t row = i / r.S_pad, s = i - row * r.S_pad;
                if (row < r.n_slots)
                    r.t32[i] = s < r.S ? static_cast<float>(r.x[row * r.S + s]) : 0.0f;
            }
        } else if (kind == SK_FINAL) {
            double *red = reinterpret_cast<double *>(lds);
            if (r.precision == COS_FP64)
                serve_final<double, KIND>(r, local, red, wave, lane);
            else if (r.precision == COS_BF16_RESCALED)
                serve_final<__bf16, KIND>(r, local, red, wave, lane);
            else if (r.precision == COS_FP16_RESCALED)
                serve_final<_Float16, KIND>(r, local, red, wave, lane);
            else
                serve_final<float, KIND>(r, local, red, wave, lane);
        } else {  // SK_COMBINE
            const int64_t s = static_cast<int64_t>(local) * kServeCombineTile + threadIdx.x;
            if (s < r.S)
                final_combine_one(reinterpret_cast<const double *>(r.ws + r.off_partial), r.final_chunks, r.S_pad, s,
                                  is_rescaled(static_cast<cos_precision>(r.precision))
                                      ? reinterpret_cast<const uint32_t *>(r.ws + r.off_maxbits)
                                      : nullptr,
                                  r.L, r.out, r.out_exp);
        }
        __syncthreads();  // LDS is reused by the group's next item
    }
}

// The step's set-up: the slot entries of the newly admitted requests, then
// their exponent rows (row 0 = row0, rows 1..L = 0), before the step kernels
// (the next graph nodes) read them.
__global__ __launch_bounds__(kBlock) void serve_setup_kernel(const StepTable *__restrict__ tab,
                                                             ServeReqDev *__restrict__ reqs) {
    static_assert(sizeof(ServeReqDev) % sizeof(uint32_t) == 0, "slot entries are copied word by word");
    constexpr uint32_t kWords = sizeof(ServeReqDev) / sizeof(uint32_t);
    const uint32_t n = tab->n_setup;
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = tid; i < static_cast<int64_t>(n) * kWords; i += stride) {
        const StepSetup &su = tab->setup[i / kWords];
        reinterpret_cast<uint32_t *>(reqs + su.slot)[i % kWords] =
            reinterpret_cast<const uint32_t *>(&su.req)[i % kWords];
    }
    for (uint32_t e = 0; e < n; ++e) {
        const StepSetup &su = tab->setup[e];
        if (!su.fill)
            continue;
        uint32_t *rows = reinterpret_cast<uint32_t *>(su.req.ws + su.req.off_maxbits);
        const int64_t total = static_cast<int64_t>(su.req.L + 1) * su.req.S_pad;
        for (int64_t i = tid; i < total; i += stride)
            rows[i] = i < su.req.S_pad ? su.row0 : 0u;
    }
}

}  // namespace

namespace {

constexpr int kServeSetupGrid = 256;

template <typename Kern>
hipError_t allow_full_lds(Kern kern) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(kLdsBytes));
}

}  // namespace

hipError_t serve_build_step_graph(StepTable *d_tab, const StepTable *h_tab, ServeReqDev *d_reqs,
                                  bool with_lookup, hipGraphExec_t *exec) {
    static std::atomic<bool> attr_set{false};
    if (!attr_set.load(std::memory_order_acquire)) {
        hipError_t err = allow_full_lds(serve_fused_kernel<FK_RATIONAL, SS_FUSED>);
        if (err == hipSuccess)
            err = allow_full_lds(serve_fused_kernel<FK_LOOKUP, SS_FUSED_LOOKUP>);
        if (err != hipSuccess)
            return err;
        attr_set.store(true, std::memory_order_release);
    }
    hipGraph_t graph = nullptr;
    hipError_t err = hipGraphCreate(&graph, 0);
    if (err != hipSuccess)
        return err;
    hipGraphNode_t upload = nullptr;
    err = hipGraphAddMemcpyNode1D(&upload, graph, nullptr, 0, d_tab, h_tab, sizeof(StepTable),
                                  hipMemcpyHostToDevice);
    const StepTable *tab_arg = d_tab;
    const ServeReqDev *reqs_arg = d_reqs;
    void *args[] = {&tab_arg, &reqs_arg};
    ServeReqDev *reqs_out = d_reqs;
    void *setup_args[] = {&tab_arg, &reqs_out};
    hipGraphNode_t setup = nullptr;
    if (err == hipSuccess) {
        hipKernelNodeParams kp{};
        kp.func = reinterpret_cast<void *>(serve_setup_kernel);
        kp.gridDim = dim3(kServeSetupGrid);
        kp.blockDim = dim3(kBlock);
        kp.kernelParams = setup_args;
        err = hipGraphAddKernelNode(&setup, graph, &upload, 1, &kp);
    }
    auto add = [&](void *func, bool fused) {
        if (err != hipSuccess)
            return;
        hipKernelNodeParams kp{};
        kp.func = func;
        kp.gridDim = dim3(fused ? kServeFusedGrid : kServeStreamGrid);
        kp.blockDim = dim3(fused ? kFusedThreads : kBlock);
        kp.sharedMemBytes = fused ? static_cast<unsigned>(kLdsBytes) : 0u;
        kp.kernelParams = args;
        hipGraphNode_t node = nullptr;
        err = hipGraphAddKernelNode(&node, graph, &setup, 1, &kp);
    };
    add(reinterpret_cast<void *>(serve_fused_kernel<FK_RATIONAL, SS_FUSED>), true);
    add(reinterpret_cast<void *>(serve_stream_kernel<FK_RATIONAL, SS_STREAMED>), false);
    if (with_lookup) {
        add(reinterpret_cast<void *>(serve_fused_kernel<FK_LOOKUP, SS_FUSED_LOOKUP>), true);
        add(reinterpret_cast<void *>(serve_stream_kernel<FK_LOOKUP, SS_STREAMED_LOOKUP>), false);
    }
    if (err == hipSuccess)
        err = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    return err;
}

}  // namespace cosdag
