// Host side of the library: errors, graph ingest (validation, canonical order,
// per-level CSR, parameter records), upload, introspection and the timing probe.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>

#include "cos_internal.h"

#ifndef COS_BUILD_ID
#define COS_BUILD_ID "unknown"
#endif

struct cos_graph {
    cosdag::Graph g;
};

namespace cosdag {

static thread_local std::string t_error;

void set_error(const std::string &msg) { t_error = msg; }

cos_status fail(cos_status st, const std::string &msg) {
    t_error = msg;
    return st;
}

cos_status hip_fail(hipError_t err, const char *what) {
    t_error = std::string(what) + ": " + hipGetErrorString(err);
    return err == hipErrorOutOfMemory ? COS_ENOMEM : COS_EDEVICE;
}

// ---------------------------------------------------------------- timing probe
namespace {
struct TimingRec {
    int kind;
    hipEvent_t start, stop;
};
std::mutex g_tmu;
std::atomic<bool> g_timing{false};  // read without the lock by launching threads
std::vector<TimingRec> g_recs;
std::vector<hipEvent_t> g_pool;
thread_local hipEvent_t t_open_start[KK_COUNT] = {};

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}
}  // namespace

bool timing_on() { return g_timing; }

void timing_begin(int kind, hipStream_t s) {
    if (!g_timing)
        return;
    std::lock_guard<std::mutex> lk(g_tmu);
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s) == hipSuccess)
        t_open_start[kind] = e;
}

void timing_end(int kind, hipStream_t s) {
    if (!g_timing || !t_open_start[kind])
        return;
    std::lock_guard<std::mutex> lk(g_tmu);
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s) == hipSuccess)
        g_recs.push_back({kind, t_open_start[kind], e});
    t_open_start[kind] = nullptr;
}

}  // namespace cosdag

using namespace cosdag;

extern "C" const char *cos_last_error(void) { return t_error.c_str(); }
extern "C" const char *cos_build_id(void) { return COS_BUILD_ID; }
extern "C" int32_t cos_abi_version(void) { return COS_ABI_VERSION; }

extern "C" cos_status cos_timing_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = enable != 0;
    return COS_OK;
}

extern "C" cos_status cos_timing_read(int32_t kind, double *total_ms, int64_t *launches) {
    if (kind < 0 || kind >= KK_COUNT || !total_ms || !launches)
        return fail(COS_EINVAL, "cos_timing_read: bad kind or NULL output");
    std::lock_guard<std::mutex> lk(g_tmu);
    double tot = 0.0;
    int64_t n = 0;
    std::vector<TimingRec> keep;
    for (const TimingRec &r : g_recs) {
        if (r.kind != kind) {
            keep.push_back(r);
            continue;
        }
        hipError_t err = hipEventSynchronize(r.stop);
        float ms = 0.f;
        if (err == hipSuccess)
            err = hipEventElapsedTime(&ms, r.start, r.stop);
        if (err != hipSuccess)
            return hip_fail(err, "cos_timing_read");
        tot += ms;
        ++n;
        g_pool.push_back(r.start);
        g_pool.push_back(r.stop);
    }
    g_recs.swap(keep);
    *total_ms = tot;
    *launches = n;
    return COS_OK;
}

// ---------------------------------------------------------------- graph ingest
namespace {

uint64_t bits_of(double v) {
    uint64_t u;
    std::memcpy(&u, &v, sizeof u);
    return u;
}

cos_status validate_shape(int32_t L, const int64_t *widths, const int64_t *epl, int64_t *n_nodes,
                          int64_t *n_edges) {
    if (L < 1)
        return fail(COS_EINVAL, "L must be >= 1");
    if (!widths || !epl)
        return fail(COS_EINVAL, "widths / edges_per_level is NULL");
    if (widths[0] != 1 || widths[L] != 1)
        return fail(COS_EINVAL, "widths[0] and widths[L] must be 1 (single root, single final node)");
    int64_t nn = 0, ne = 0;
    for (int32_t l = 0; l <= L; ++l) {
        if (widths[l] < 1)
            return fail(COS_EINVAL, "widths[" + std::to_string(l) + "] < 1");
        nn += widths[l];
        if (nn >= INT32_MAX)
            return fail(COS_EINVAL, "node count must be < 2^31");
    }
    for (int32_t l = 0; l < L; ++l) {
        if (epl[l] < 0)
            return fail(COS_EINVAL, "edges_per_level[" + std::to_string(l) + "] < 0");
        ne += epl[l];
        if (ne >= INT32_MAX)
            return fail(COS_EINVAL, "edge count must be < 2^31");
    }
    *n_nodes = nn;
    *n_edges = ne;
    return COS_OK;
}

}  // namespace

namespace {

// Edge parameters of one of the two factor kinds.
// Headroom exponents of binary16 level storage.  Rational factors satisfy
// |w_e| <= |a_e| (the denominator is at least 1), so a level-l value is at
// most R_l = max_j sum_{e into j} |a_e| times the largest value of level l-1.
// The sweep normalises level l-1 to [1, 2) and stores level l times 2^-h_l
// with h_l = max(0, ceil(log2 R_l) - 14): every stored value stays below
// 2^15 (binary16 holds up to 65504).  Empty when some h_l would exceed
// kMaxHeadroom16 (binary16 storage is then refused).
std::vector<int32_t> headroom16(const Graph &G, const std::vector<int32_t> &row_ptr) {
    std::vector<int32_t> h(static_cast<size_t>(G.L), 0);
    for (int32_t l = 1; l <= G.L - 1; ++l) {
        const LevelDesc &d = G.levels[l - 1];
        const int32_t *r = row_ptr.data() + d.rp_begin;
        double R = 0.0;
        for (int64_t j = 0; j < d.w_dst; ++j) {
            double sum = 0.0;
            for (int64_t q = r[j]; q < r[j + 1]; ++q)
                sum += std::fabs(G.h_a[q]);
            R = std::max(R, sum);
        }
        if (!std::isfinite(R))
            return {};
        if (R > 0.0) {
            int e = 0;
            const double f = std::frexp(R, &e);  // R = f 2^e, f in [0.5, 1)
            const int c = f == 0.5 ? e - 1 : e;  // ceil(log2 R)
            h[l] = std::max(0, c - 14);
            if (h[l] > kMaxHeadroom16)
                return {};
        }
    }
    return h;
}

struct EdgeParams {
    int32_t kind = FK_RATIONAL;
    const double *a = nullptr, *b = nullptr, *k = nullptr;  // rational
    const int32_t *slot = nullptr;                           // lookup
    const double *coef = nullptr;
    int32_t n_slots = 0;
};

cos_status build_graph(int32_t L, const int64_t *widths, const int64_t *edges_per_level, const int32_t *src,
                       const int32_t *dst, const EdgeParams &P, cos_graph **out) {
    if (!out)
        return fail(COS_EINVAL, "out is NULL");
    *out = nullptr;
    int64_t n_nodes = 0, n_edges = 0;
    cos_status st = validate_shape(L, widths, edges_per_level, &n_nodes, &n_edges);
    if (st != COS_OK)
        return st;
    const bool lookup = P.kind == FK_LOOKUP;
    if (lookup && P.n_slots < 1)
        return fail(COS_EINVAL, "n_slots must be >= 1");
    if (n_edges > 0 && (!src || !dst || (lookup ? (!P.slot || !P.coef) : (!P.a || !P.b || !P.k))))
        return fail(COS_EINVAL, "edge arrays are NULL");

    auto h = std::make_unique<cos_graph>();
    Graph &G = h->g;
    G.kind = P.kind;
    G.n_slots = lookup ? P.n_slots : 0;
    G.L = L;
    G.widths.assign(widths, widths + L + 1);
    G.level_first.resize(L + 2);
    G.level_first[0] = 0;
    for (int32_t l = 0; l <= L; ++l)
        G.level_first[l + 1] = G.level_first[l] + widths[l];
    G.n_nodes = n_nodes;
    G.n_edges = n_edges;

    // validate every edge against its level and its parameters
    int64_t e = 0;
    for (int32_t l = 1; l <= L; ++l) {
        const int64_t s_lo = G.level_first[l - 1], s_hi = G.level_first[l];
        const int64_t d_lo = G.level_first[l], d_hi = G.level_first[l + 1];
        for (int64_t i = 0; i < edges_per_level[l - 1]; ++i, ++e) {
            if (src[e] < s_lo || src[e] >= s_hi || dst[e] < d_lo || dst[e] >= d_hi)
                return fail(COS_EINVAL, "edge " + std::to_string(e) + " (" + std::to_string(src[e]) + "->" +
                                            std::to_string(dst[e]) + ") does not join level " +
                                            std::to_string(l - 1) + " to level " + std::to_string(l));
            if (lookup) {
                if (P.slot[e] < 0 || P.slot[e] >= P.n_slots || !std::isfinite(P.coef[e]))
                    return fail(COS_EINVAL, "edge " + std::to_string(e) +
                                                ": slot must be in 0..n_slots-1 and the constant finite");
            } else if (!std::isfinite(P.a[e]) || !std::isfinite(P.b[e]) || P.b[e] < 0.0 ||
                       !std::isfinite(P.k[3 * e]) || !std::isfinite(P.k[3 * e + 1]) ||
                       !std::isfinite(P.k[3 * e + 2])) {
                return fail(COS_EINVAL, "edge " + std::to_string(e) + ": parameters must be finite with b >= 0");
            } else {
                // the expanded binary64 denominator c0 + b|x|^2 + g.x (c0 = 1 + b|k|^2,
                // g = -2bk) is what the binary64 sweep and every final node evaluate:
                // its coefficients must be finite
                const double b = P.b[e], k0 = P.k[3 * e], k1 = P.k[3 * e + 1], k2 = P.k[3 * e + 2];
                if (!std::isfinite(1.0 + b * (k0 * k0 + k1 * k1 + k2 * k2)) || !std::isfinite(2.0 * b * k0) ||
                    !std::isfinite(2.0 * b * k1) || !std::isfinite(2.0 * b * k2))
                    return fail(COS_EINVAL, "edge " + std::to_string(e) + ": 1 + b|k|^2 or 2bk overflows binary64");
            }
        }
    }

    // canonical order within each level: (dst, src, then the parameters:
    // bits of a, b, k0, k1, k2 -- or the slot and the bits of the constant)
    std::vector<int64_t> order(n_edges);
    std::iota(order.begin(), order.end(), 0);
    G.levels.resize(L);
    int64_t e0 = 0, rp = 0;
    for (int32_t l = 1; l <= L; ++l) {
        const int64_t ne = edges_per_level[l - 1];
        auto less = [&](int64_t i, int64_t j) {
            if (dst[i] != dst[j])
                return dst[i] < dst[j];
            if (src[i] != src[j])
                return src[i] < src[j];
            if (lookup) {
                if (P.slot[i] != P.slot[j])
                    return P.slot[i] < P.slot[j];
                return bits_of(P.coef[i]) < bits_of(P.coef[j]);
            }
            const double pi[5] = {P.a[i], P.b[i], P.k[3 * i], P.k[3 * i + 1], P.k[3 * i + 2]};
            const double pj[5] = {P.a[j], P.b[j], P.k[3 * j], P.k[3 * j + 1], P.k[3 * j + 2]};
            for (int c = 0; c < 5; ++c)
                if (bits_of(pi[c]) != bits_of(pj[c]))
                    return bits_of(pi[c]) < bits_of(pj[c]);
            return false;
        };
        std::sort(order.begin() + e0, order.begin() + e0 + ne, less);
        LevelDesc &d = G.levels[l - 1];
        d.w_src = widths[l - 1];
        d.w_dst = widths[l];
        d.e_begin = e0;
        d.n_edges = ne;
        d.rp_begin = rp;
        rp += d.w_dst + 1;
        e0 += ne;
    }

    G.h_src.resize(n_edges);
    G.h_dst.resize(n_edges);
    if (lookup) {
        G.h_slot.resize(n_edges);
        G.h_coef.resize(n_edges);
    } else {
        G.h_a.resize(n_edges);
        G.h_b.resize(n_edges);
        G.h_k.resize(3 * n_edges);
    }
    for (int64_t i = 0; i < n_edges; ++i) {
        const int64_t o = order[i];
        G.h_src[i] = src[o];
        G.h_dst[i] = dst[o];
        if (lookup) {
            G.h_slot[i] = P.slot[o];
            G.h_coef[i] = P.coef[o];
        } else {
            G.h_a[i] = P.a[o];
            G.h_b[i] = P.b[o];
            G.h_k[3 * i] = P.k[3 * o];
            G.h_k[3 * i + 1] = P.k[3 * o + 1];
            G.h_k[3 * i + 2] = P.k[3 * o + 2];
        }
    }
    order.clear();
    order.shrink_to_fit();

    // per-level CSR over destinations (global edge indices) and edge records
    std::vector<int32_t> row_ptr(rp);
    std::vector<EdgeRec> recs(lookup ? 0 : n_edges + kEdgePad, EdgeRec{});
    std::vector<EdgeRec32> recs32(lookup ? 0 : n_edges + kEdgePad, EdgeRec32{});
    std::vector<EdgeRecL> recsL(lookup ? n_edges + kEdgePad : 0, EdgeRecL{});
    std::vector<LevelDev> ldev(L);
    std::vector<int32_t> hub_chunks;  // (first edge, end edge) pairs
    for (int32_t l = 1; l <= L; ++l) {
        LevelDesc &d = G.levels[l - 1];
        int32_t *r = row_ptr.data() + d.rp_begin;
        const int64_t dfirst = G.level_first[l], sfirst = G.level_first[l - 1];
        int64_t i = d.e_begin, maxdeg = 0;
        for (int64_t j = 0; j < d.w_dst; ++j) {
            r[j] = static_cast<int32_t>(i);
            const int64_t start = i;
            while (i < d.e_begin + d.n_edges && G.h_dst[i] == dfirst + j)
                ++i;
            maxdeg = std::max(maxdeg, i - start);
        }
        r[d.w_dst] = static_cast<int32_t>(i);
        d.max_deg = maxdeg;
        if (l < L) {
            G.max_width = std::max(G.max_width, d.w_dst);
            G.max_in_degree = std::max(G.max_in_degree, maxdeg);
        }
        for (int64_t q = d.e_begin; q < d.e_begin + d.n_edges; ++q) {
            const int32_t src_local = static_cast<int32_t>(G.h_src[q] - sfirst);
            if (lookup) {
                EdgeRecL &rl = recsL[q];
                rl.coef = G.h_coef[q];
                rl.coef32 = static_cast<float>(G.h_coef[q]);
                G.f32_ok = G.f32_ok && std::isfinite(rl.coef32);
                rl.slot = G.h_slot[q];
                rl.src = src_local;
                continue;
            }
            const double b = G.h_b[q], k0 = G.h_k[3 * q], k1 = G.h_k[3 * q + 1], k2 = G.h_k[3 * q + 2];
            EdgeRec &rec = recs[q];
            rec.c0 = 1.0 + b * (k0 * k0 + k1 * k1 + k2 * k2);
            rec.cb = b;
            rec.g0 = -2.0 * b * k0;
            rec.g1 = -2.0 * b * k1;
            rec.g2 = -2.0 * b * k2;
            rec.a = G.h_a[q];
            rec.src = src_local;
            EdgeRec32 &r32 = recs32[q];
            r32.a = static_cast<float>(G.h_a[q]);
            r32.b = static_cast<float>(b);
            r32.k0 = static_cast<float>(k0);
            r32.k1 = static_cast<float>(k1);
            r32.k2 = static_cast<float>(k2);
            r32.src = src_local;
            G.f32_ok = G.f32_ok && std::isfinite(r32.a) && std::isfinite(r32.b) && std::isfinite(r32.k0) &&
                       std::isfinite(r32.k1) && std::isfinite(r32.k2);
        }
        // row boundaries inside the edge stream: the last edge of every
        // non-empty row, and how many empty rows follow it
        for (int64_t j = 0; j < d.w_dst; ++j) {
            if (r[j + 1] == r[j])
                continue;
            int64_t z = j + 1;
            while (z < d.w_dst && r[z + 1] == r[z])
                ++z;
            const int64_t last = r[j + 1] - 1;
            const int32_t zr = static_cast<int32_t>(z - (j + 1));
            if (lookup) {
                recsL[last].row_end = 1;
                recsL[last].zero_rows = zr;
            } else {
                recs[last].row_end = 1;
                recs[last].zero_rows = zr;
                recs32[last].row_end = 1;
                recs32[last].zero_rows = zr;
            }
        }
        // rows of high in-degree (interior levels): their chunk lists, and the
        // index of each such row's first chunk in the row's first record
        if (l < L) {
            d.hub_begin = static_cast<int64_t>(hub_chunks.size() / 2);
            for (int64_t j = 0; j < d.w_dst; ++j) {
                const int64_t e_lo = r[j], e_hi = r[j + 1];
                if (e_hi - e_lo <= kHubEdges)
                    continue;
                const int32_t first = static_cast<int32_t>(hub_chunks.size() / 2 - d.hub_begin);
                if (lookup)
                    recsL[e_lo].zero_rows = first;
                else {
                    recs[e_lo].zero_rows = first;
                    recs32[e_lo].zero_rows = first;
                }
                for (int64_t c = e_lo; c < e_hi; c += kFinalChunk) {
                    hub_chunks.push_back(static_cast<int32_t>(c));
                    hub_chunks.push_back(static_cast<int32_t>(std::min<int64_t>(c + kFinalChunk, e_hi)));
                }
            }
            d.n_hub_chunks = static_cast<int64_t>(hub_chunks.size() / 2) - d.hub_begin;
            G.max_hub_chunks = std::max(G.max_hub_chunks, d.n_hub_chunks);
        }
        ldev[l - 1] = LevelDev{static_cast<int32_t>(d.w_dst), static_cast<int32_t>(d.rp_begin),
                               static_cast<int32_t>(d.e_begin), static_cast<int32_t>(d.n_edges),
                               d.n_hub_chunks > 0 ? 1 : 0, {0, 0, 0}};
    }
    if (!lookup)
        G.h16 = headroom16(G, row_ptr);

    // panel plan of wide graphs without rows of high in-degree: each
    // interior level's rows in two halves of about equal edge counts, each half
    // cut into panels of consecutive rows whose records and row offsets fit
    // the LDS budget, at least 32 per half (one per CU of an XCD) and a
    // multiple of 32, of about equal edge counts
    std::vector<int32_t> panels;  // (first row, end row, first edge, end edge)
    // (a source's byte offset within a tile of the level must fit 32 bits)
    G.panel_ok = G.max_hub_chunks == 0 && G.max_width >= kPanelMinWidth &&
                 G.max_width < (int64_t{1} << 24) && L >= 2;
    for (int32_t l = 1; l < L && G.panel_ok; ++l) {
        LevelDesc &d = G.levels[l - 1];
        const int32_t *r = row_ptr.data() + d.rp_begin;
        const int64_t W = d.w_dst;
        d.panel_begin = static_cast<int64_t>(panels.size() / 4);
        // the first half ends at the first row where half of the level's edges are reached
        int64_t mid = 0;
        while (mid < W && 2 * (static_cast<int64_t>(r[mid]) - r[0]) < d.n_edges)
            ++mid;
        mid = W > 1 ? std::min<int64_t>(std::max<int64_t>(mid, 1), W - 1) : W;
        const int64_t halves[3] = {0, mid, W};
        for (int h = 0; h < 2; ++h) {
            const int64_t r0 = halves[h], r1 = halves[h + 1];
            if (r1 <= r0)
                continue;
            const int64_t ne = static_cast<int64_t>(r[r1]) - r[r0];
            const int64_t bytes = (ne + kPanelPadRecs) * 24 + (r1 - r0 + 1) * 4;
            int64_t n = std::max<int64_t>(32, (bytes + kPanelRecBytes - 1) / kPanelRecBytes);
            n = (n + 31) / 32 * 32;
            const int64_t target = std::max<int64_t>(1, (ne + n - 1) / n);
            int64_t pr = r0;
            while (pr < r1) {
                int64_t q = pr, e_in = 0;
                while (q < r1) {
                    const int64_t deg = static_cast<int64_t>(r[q + 1]) - r[q];
                    const int64_t need = round_up((e_in + deg + kPanelPadRecs) * 24 + (q - pr + 2) * 4, 16);
                    if (q > pr && (e_in + deg > target || need > kPanelRecBytes || q - pr >= kPanelMaxRows))
                        break;
                    e_in += deg;
                    ++q;
                }
                const int64_t need = round_up((e_in + kPanelPadRecs) * 24 + (q - pr + 1) * 4, 16);
                if (need > kPanelRecBytes) {  // one row alone exceeds the budget
                    G.panel_ok = false;
                    break;
                }
                d.panel_lds = std::max(d.panel_lds, kPanelSampleBytes + need);
                panels.insert(panels.end(), {static_cast<int32_t>(pr), static_cast<int32_t>(q), r[pr], r[q]});
                pr = q;
            }
            if (h == 0)
                d.n_panel_half0 = static_cast<int64_t>(panels.size() / 4) - d.panel_begin;
        }
        d.n_panels = static_cast<int64_t>(panels.size() / 4) - d.panel_begin;
    }
    if (!G.panel_ok)
        panels.clear();

    // one device allocation: row_ptr | edge record arrays | level table
    const size_t off_rp = 0;
    const size_t off_rec = round_up(rp * sizeof(int32_t), 256);
    const size_t off_rec32 = off_rec + round_up(recs.size() * sizeof(EdgeRec), 256);
    const size_t off_recL = off_rec32 + round_up(recs32.size() * sizeof(EdgeRec32), 256);
    const size_t off_lev = off_recL + round_up(recsL.size() * sizeof(EdgeRecL), 256);
    const size_t off_h16 = off_lev + round_up(L * sizeof(LevelDev), 256);
    const size_t off_hub = off_h16 + round_up(G.h16.size() * sizeof(int32_t), 256);
    const size_t off_panel = off_hub + round_up(hub_chunks.size() * sizeof(int32_t), 256);
    const size_t total = off_panel + round_up(panels.size() * sizeof(int32_t), 256);
    hipError_t err = hipGetDevice(&G.device);
    if (err != hipSuccess)
        return hip_fail(err, "hipGetDevice");
    err = hipMalloc(&G.d_base, total);
    if (err != hipSuccess)
        return hip_fail(err, "hipMalloc(graph)");
    G.d_bytes = total;
    char *base = static_cast<char *>(G.d_base);
    G.d_row_ptr = reinterpret_cast<int32_t *>(base + off_rp);
    G.d_edges = lookup ? nullptr : reinterpret_cast<EdgeRec *>(base + off_rec);
    G.d_edges32 = lookup ? nullptr : reinterpret_cast<EdgeRec32 *>(base + off_rec32);
    G.d_edgesL = lookup ? reinterpret_cast<EdgeRecL *>(base + off_recL) : nullptr;
    G.d_levels = reinterpret_cast<LevelDev *>(base + off_lev);
    G.d_h16 = G.h16.empty() ? nullptr : reinterpret_cast<int32_t *>(base + off_h16);
    G.d_hub_chunks = hub_chunks.empty() ? nullptr : reinterpret_cast<int32_t *>(base + off_hub);
    G.d_panels = panels.empty() ? nullptr : reinterpret_cast<int32_t *>(base + off_panel);
    err = hipMemcpy(G.d_row_ptr, row_ptr.data(), rp * sizeof(int32_t), hipMemcpyHostToDevice);
    if (err == hipSuccess && !recs.empty())
        err = hipMemcpy(G.d_edges, recs.data(), recs.size() * sizeof(EdgeRec), hipMemcpyHostToDevice);
    if (err == hipSuccess && !recs32.empty())
        err = hipMemcpy(G.d_edges32, recs32.data(), recs32.size() * sizeof(EdgeRec32), hipMemcpyHostToDevice);
    if (err == hipSuccess && !recsL.empty())
        err = hipMemcpy(G.d_edgesL, recsL.data(), recsL.size() * sizeof(EdgeRecL), hipMemcpyHostToDevice);
    if (err == hipSuccess)
        err = hipMemcpy(G.d_levels, ldev.data(), L * sizeof(LevelDev), hipMemcpyHostToDevice);
    if (err == hipSuccess && G.d_h16)
        err = hipMemcpy(G.d_h16, G.h16.data(), G.h16.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (err == hipSuccess && G.d_panels)
        err = hipMemcpy(G.d_panels, panels.data(), panels.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (err == hipSuccess && G.d_hub_chunks)
        err = hipMemcpy(G.d_hub_chunks, hub_chunks.data(), hub_chunks.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        (void)hipFree(G.d_base);
        return hip_fail(err, "hipMemcpy(graph)");
    }
    *out = h.release();
    return COS_OK;
}

}  // namespace

extern "C" cos_status cos_create_graph(int32_t L, const int64_t *widths, const int64_t *edges_per_level,
                                       const int32_t *src, const int32_t *dst, const double *a,
                                       const double *b, const double *k, cos_graph **out) {
    try {
        EdgeParams P;
        P.kind = FK_RATIONAL;
        P.a = a;
        P.b = b;
        P.k = k;
        return build_graph(L, widths, edges_per_level, src, dst, P, out);
    } catch (const std::bad_alloc &) {
        return fail(COS_ENOMEM, "host allocation failed in cos_create_graph");
    } catch (...) {
        return fail(COS_EDEVICE, "unexpected exception in cos_create_graph");
    }
}

extern "C" cos_status cos_create_graph_lookup(int32_t L, const int64_t *widths, const int64_t *edges_per_level,
                                              const int32_t *src, const int32_t *dst, const int32_t *slot,
                                              const double *coef, int32_t n_slots, cos_graph **out) {
    try {
        EdgeParams P;
        P.kind = FK_LOOKUP;
        P.slot = slot;
        P.coef = coef;
        P.n_slots = n_slots;
        return build_graph(L, widths, edges_per_level, src, dst, P, out);
    } catch (const std::bad_alloc &) {
        return fail(COS_ENOMEM, "host allocation failed in cos_create_graph_lookup");
    } catch (...) {
        return fail(COS_EDEVICE, "unexpected exception in cos_create_graph_lookup");
    }
}

extern "C" cos_status cos_graph_get_info(const cos_graph *h, cos_graph_info *info) {
    if (!h || !info)
        return fail(COS_EINVAL, "cos_graph_get_info: NULL argument");
    const Graph &G = h->g;
    info->L = G.L;
    info->fused_mask = (fused_fits(G, COS_FP64) ? 1 : 0) | (fused_fits(G, COS_FP32_RESCALED) ? 2 : 0) |
                       (fused_fits(G, COS_FP32) ? 4 : 0);
    info->panel_mask = 0;
    for (const cos_precision p : {COS_FP64, COS_FP32_RESCALED, COS_FP32, COS_FP16_RESCALED, COS_BF16_RESCALED})
        info->panel_mask |= panel_fits(G, p) ? 1 << p : 0;
    info->reserved = 0;
    info->n_nodes = G.n_nodes;
    info->n_edges = G.n_edges;
    info->max_width = G.max_width;
    info->max_in_degree = G.max_in_degree;
    info->final_in_degree = G.levels.back().n_edges;
    info->device_bytes = G.d_bytes;
    info->factor_kind = G.kind;
    info->n_inputs = G.kind == FK_LOOKUP ? G.n_slots : 3;
    return COS_OK;
}

extern "C" cos_status cos_graph_set_path(cos_graph *h, cos_path path) {
    if (!h)
        return fail(COS_EINVAL, "cos_graph_set_path: graph is NULL");
    if (path != COS_PATH_AUTO && path != COS_PATH_STREAMED && path != COS_PATH_FUSED && path != COS_PATH_PANEL)
        return fail(COS_EINVAL, "cos_graph_set_path: unknown path");
    h->g.path = path;
    return COS_OK;
}

extern "C" cos_status cos_graph_export(const cos_graph *h, int32_t *src, int32_t *dst, double *a, double *b,
                                       double *k) {
    if (!h || !src || !dst || !a || !b || !k)
        return fail(COS_EINVAL, "cos_graph_export: NULL argument");
    const Graph &G = h->g;
    if (G.kind != FK_RATIONAL)
        return fail(COS_EINVAL, "cos_graph_export: the graph has lookup factors (use cos_graph_export_lookup)");
    const size_t n = static_cast<size_t>(G.n_edges);
    std::memcpy(src, G.h_src.data(), n * sizeof(int32_t));
    std::memcpy(dst, G.h_dst.data(), n * sizeof(int32_t));
    std::memcpy(a, G.h_a.data(), n * sizeof(double));
    std::memcpy(b, G.h_b.data(), n * sizeof(double));
    std::memcpy(k, G.h_k.data(), 3 * n * sizeof(double));
    return COS_OK;
}

extern "C" cos_status cos_graph_export_lookup(const cos_graph *h, int32_t *src, int32_t *dst, int32_t *slot,
                                              double *coef) {
    if (!h || !src || !dst || !slot || !coef)
        return fail(COS_EINVAL, "cos_graph_export_lookup: NULL argument");
    const Graph &G = h->g;
    if (G.kind != FK_LOOKUP)
        return fail(COS_EINVAL, "cos_graph_export_lookup: the graph has rational factors (use cos_graph_export)");
    const size_t n = static_cast<size_t>(G.n_edges);
    std::memcpy(src, G.h_src.data(), n * sizeof(int32_t));
    std::memcpy(dst, G.h_dst.data(), n * sizeof(int32_t));
    std::memcpy(slot, G.h_slot.data(), n * sizeof(int32_t));
    std::memcpy(coef, G.h_coef.data(), n * sizeof(double));
    return COS_OK;
}

extern "C" cos_status cos_destroy_graph(cos_graph *h) {
    if (!h)
        return COS_OK;
    hipError_t err = h->g.d_base ? hipFree(h->g.d_base) : hipSuccess;
    delete h;
    if (err != hipSuccess)
        return hip_fail(err, "hipFree(graph)");
    return COS_OK;
}

// accessor for the other translation units
namespace cosdag {
const Graph &graph_of(const cos_graph *h) { return h->g; }

cos_status check_precision_range(const Graph &g, cos_precision p, const char *who) {
    if (p != COS_FP64 && !g.f32_ok)
        return fail(COS_EINVAL, std::string(who) + ": an edge parameter lies beyond the binary32 range (it rounds "
                                                   "to infinity); evaluate this graph with COS_FP64");
    return COS_OK;
}
}  // namespace cosdag
