// HIP kernels of the bake (Eq. 6 with the Fresnel split of Eq. 7 and the
// stage-1 radiance query of Eq. 9) and of shading-point generation, for
// gfx950.
//
// Mapping: one wavefront bakes one point; its 64 lanes take 64 consecutive
// (lobe, sample) pairs of that point, flattened over the diffuse lobe and
// the K specular levels, so the lanes of a wave share the ray origin and
// start traversal on the same nodes.  After each chunk of 64 samples the
// contributions of every lobe present in the chunk are summed by a fixed
// xor butterfly; each lane keeps the running sums of two accumulator slots
// in registers.  The summation order depends only on the sample counts, so
// a point's result is bitwise independent of which launch, tile or batch it
// was baked in.
//
// Traversal stacks live in LDS, 32 entries per lane, lane-minor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>

#include "device.hpp"
#include "fipt_internal.hpp"

namespace fipt {
namespace {

using dev::V3;
using dev::v3;
using dev::lobe_of;
using dev::next_point;
using dev::slot_plane;
using dev::wave_uniform;

constexpr int kBlock = 64;              // one wavefront: a finished wave frees its LDS at once
constexpr int kWaves = kBlock / 64;
// persistent grids: one round of the 20 wavefronts a CU holds at once (5
// per SIMD at 96 VGPRs, 8 KB of LDS each); points are handed out
// dynamically, so a larger grid only queues workgroups, and the server's
// back-to-back launches on two streams then crowd each other
constexpr int kGridWavesPerCu = 20;

// Bake point p of job b with the calling wavefront.
template <bool COUNT, bool VOXEL>
__device__ __forceinline__ void bake_point(const BakeLaunch& b, const float* sigma, int64_t p, int lane,
                                           int32_t* stack, uint32_t& n_rays, uint32_t& n_nodes,
                                           uint32_t& n_tris, uint32_t& n_hits) {
    const int K = b.K;
    const int P = 3 + 6 * K;
    const int64_t ps = b.pts_stride;
    const int32_t tri = b.ptri[p];
    V3 x = v3(b.pts[p], b.pts[ps + p], b.pts[2 * ps + p]);
    V3 n = v3(b.pts[3 * ps + p], b.pts[4 * ps + p], b.pts[5 * ps + p]);
    const V3 wo = v3(b.pts[6 * ps + p], b.pts[7 * ps + p], b.pts[8 * ps + p]);
    float cos_o = dev::dot(n, wo);
    if (tri >= 0 && cos_o < 0.0f) {
        n = v3(-n.x, -n.y, -n.z);
        cos_o = -cos_o;
    }
    const int64_t os = b.out_stride;
    if (!(tri >= 0 && cos_o > 0.0f)) {
        for (int j = lane; j < P; j += 64) b.out[(int64_t)j * os + p] = 0.0f;
        return;
    }
    V3 ft, fb;
    dev::make_frame(n, ft, fb);
    const V3 o = x + b.eps * n;
    const int64_t rng_p = p + b.p_offset;
    const int spp_d = b.spp_d, spp_s = b.spp_s;
    const int S = spp_d + K * spp_s;
    float acc_a = 0.0f, acc_b = 0.0f;   // slots lane and 64 + lane
    for (int q0 = 0; q0 < S; q0 += 64) {
        const int q = q0 + lane;
        const bool active = q < S;
        const int lobe = active ? lobe_of(q, spp_d, spp_s) : -1;
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, c3 = 0.0f, c4 = 0.0f, c5 = 0.0f;
        V3 wi = v3(0.0f, 0.0f, 1.0f);
        float w = 0.0f, F1 = 0.0f;
        bool shoot = false;
        if (active) {
            const int s = lobe == 0 ? q : (q - spp_d) - (lobe - 1) * spp_s;
            float xi1, xi2;
            dev::lobe_uniforms(b.seed, rng_p, lobe, s, lobe == 0 ? b.w_d : b.w_s, xi1, xi2);
            float sp_, cp_;
            // azimuth 2 pi xi2: the hardware sine and cosine take the angle
            // in turns (within 1.2e-7 of sincospif for every 24-bit xi2)
            sp_ = __builtin_amdgcn_sinf(xi2);
            cp_ = __builtin_amdgcn_cosf(xi2);
            if (lobe == 0) {
                // cosine-weighted direction; estimator weight 1
                const float r = dev::sqrt_hw(xi1);
                wi = dev::to_world(ft, fb, n, r * cp_, r * sp_, dev::sqrt_hw(1.0f - xi1));
                w = 1.0f;
                shoot = true;
            } else {
                // GGX half vector, density D(m)(n.m), alpha = sigma^2
                const float sg = sigma[lobe - 1];
                const float alpha = sg * sg;
                const float a2 = alpha * alpha;
                const float tan2 = a2 * xi1 * dev::rcp(1.0f - xi1);
                const float cos_m = dev::rsq_ge1(1.0f + tan2);
                const float sin_m = dev::sqrt_hw(tan2) * cos_m;   // accurate for tiny tilts
                const V3 m = dev::to_world(ft, fb, n, sin_m * cp_, sin_m * sp_, cos_m);
                const float om = dev::dot(wo, m);
                if (om > 0.0f) {
                    wi = (2.0f * om) * m - wo;
                    const float ci = dev::dot(n, wi);
                    if (ci > 0.0f) {
                        const float G = dev::smith_g1(a2, ci) * dev::smith_g1(a2, cos_o);
                        w = G * om * dev::rcp(cos_o * cos_m);
                        const float f = 1.0f - om;
                        const float f2 = f * f;
                        F1 = f2 * f2 * f;
                        shoot = true;
                    }
                }
            }
        }
        dev::Hit h;
        h.leaf = -1;
        h.u = h.v = 0.0f;
        if (shoot) {
            if (COUNT) ++n_rays;
            h = dev::trace<COUNT>(b.sc, o, wi, stack, kBlock, n_nodes, n_tris);
            if (COUNT && h.leaf >= 0) ++n_hits;
            const V3 R = VOXEL ? dev::radiance_voxel(b.sc, h, o, wi) : dev::radiance(b.sc, h);
            if (lobe == 0) {
                c0 = R.x;
                c1 = R.y;
                c2 = R.z;
            } else {
                const float w0 = w * (1.0f - F1), w1 = w * F1;
                c0 = R.x * w0;
                c1 = R.y * w0;
                c2 = R.z * w0;
                c3 = R.x * w1;
                c4 = R.y * w1;
                c5 = R.z * w1;
            }
        }
        // reduce every lobe present in this chunk
        const int l_first = lobe_of(q0, spp_d, spp_s);
        const int l_last = lobe_of(min(q0 + 63, S - 1), spp_d, spp_s);
        for (int l = l_first; l <= l_last; ++l) {
            const bool mine = lobe == l;
            const float r0 = dev::wave_sum(mine ? c0 : 0.0f);
            const float r1 = dev::wave_sum(mine ? c1 : 0.0f);
            const float r2 = dev::wave_sum(mine ? c2 : 0.0f);
            const int base = l == 0 ? 0 : 3 + 6 * (l - 1);
            float r3 = 0.0f, r4 = 0.0f, r5 = 0.0f;
            if (l > 0) {
                r3 = dev::wave_sum(mine ? c3 : 0.0f);
                r4 = dev::wave_sum(mine ? c4 : 0.0f);
                r5 = dev::wave_sum(mine ? c5 : 0.0f);
            }
            const int na = lane - base, nb = lane + 64 - base;
            const float ra = na == 0 ? r0 : na == 1 ? r1 : na == 2 ? r2 : na == 3 ? r3 : na == 4 ? r4 : r5;
            const float rb = nb == 0 ? r0 : nb == 1 ? r1 : nb == 2 ? r2 : nb == 3 ? r3 : nb == 4 ? r4 : r5;
            const int width = l == 0 ? 3 : 6;
            if (na >= 0 && na < width) acc_a += ra;
            if (nb >= 0 && nb < width) acc_b += rb;
        }
    }
    if (lane < P) {
        const float cnt = lane < 3 ? (float)spp_d : (float)spp_s;
        b.out[(int64_t)slot_plane(lane, K) * os + p] = acc_a / cnt;
    }
    if (64 + lane < P) {
        b.out[(int64_t)slot_plane(64 + lane, K) * os + p] = acc_b / (float)spp_s;
    }
}

// ---------------------------------------------------------------------------
// Bake of one point with dynamic sample refill (K <= kRefillMaxK).
//
// The chunked bake above keeps a lane idle from the moment its ray finishes
// until the slowest ray of its 64-sample chunk does; with incoherent rays
// the slowest is several times the average.  Here every lane owns one ray
// at a time and, once a batch of lanes has finished, those lanes fold their
// results into per-lane accumulators and take the next samples of the point
// (handed out in lane order by a ballot, so the assignment depends only on
// the inputs).  Traversal is while-while with speculation: a lane that
// reaches a leaf parks it and keeps descending while other lanes are still
// looking for theirs; once only a few lanes are still searching, all lanes
// test their parked leaves together.
// At the end of the point one fixed butterfly sums the accumulators.
constexpr int kRefillMaxK = 10;      // 3 + 6K output slots fit the 64 lanes
using dev::kDone;
constexpr int kRefillMin = 40;       // refill once this many lanes are free
constexpr int kSearchMin = 10;       // leave the node loop below this many searchers

enum LaneState { kIdle = 0, kTracing = 1, kFinished = 2 };

// A leaf reference: negative but not kDone (INT_MIN).  No leaf encodes to
// INT_MIN, which would need first = 2^28 - 1 with 8 triangles.
__device__ __forceinline__ bool is_leaf(int32_t ref) {
    return (uint32_t)ref > (uint32_t)kDone;
}

template <bool COUNT, bool VOXEL>
__device__ __forceinline__ void bake_point_refill(const BakeLaunch& b, const float* sigma, int64_t p,
                                                  int lane,
                                                  int32_t* stack, uint32_t& n_rays,
                                                  uint32_t& n_nodes, uint32_t& n_tris,
                                                  uint32_t& n_hits, uint32_t& n_node_steps,
                                                  uint32_t& n_tri_steps, uint32_t& n_chain) {
    const int K = b.K;
    const int P = 3 + 6 * K;
    const int64_t ps = b.pts_stride;
    const int32_t tri = b.ptri[p];
    V3 x = v3(b.pts[p], b.pts[ps + p], b.pts[2 * ps + p]);
    V3 n = v3(b.pts[3 * ps + p], b.pts[4 * ps + p], b.pts[5 * ps + p]);
    const V3 wo = v3(b.pts[6 * ps + p], b.pts[7 * ps + p], b.pts[8 * ps + p]);
    float cos_o = dev::dot(n, wo);
    if (tri >= 0 && cos_o < 0.0f) {
        n = v3(-n.x, -n.y, -n.z);
        cos_o = -cos_o;
    }
    const int64_t os = b.out_stride;
    if (!(tri >= 0 && cos_o > 0.0f)) {
        for (int j = lane; j < P; j += 64) b.out[(int64_t)j * os + p] = 0.0f;
        return;
    }
    V3 ft, fb;
    dev::make_frame(n, ft, fb);
    const V3 o = x + b.eps * n;
    const int64_t rng_p = p + b.p_offset;
    const int spp_d = b.spp_d, spp_s = b.spp_s;
    const int S = spp_d + K * spp_s;
    const DeviceScene& sc = b.sc;
    // the boxes around o that every ray of the point enters first
    int32_t chain, chain_end;
    const int chain_len = dev::point_chain(sc.nodes, sc.box_scale, o, lane, chain, chain_end);

    // Lane j owns output slot j (slot layout as slot_plane).  Each lane sums
    // its contributions for its current lobe in cur[]; a lane's lobes only
    // increase (samples are handed out in order), so when it moves on, its
    // partial sums for the old lobe are flushed: all lanes leaving the same
    // lobe at once are summed by the fixed butterfly and the owners add the
    // totals.  Everything depends only on the inputs, so results are
    // reproducible bit for bit.
    float own = 0.0f;
    float cur0 = 0.0f, cur1 = 0.0f, cur2 = 0.0f, cur3 = 0.0f, cur4 = 0.0f, cur5 = 0.0f;
    int cur_lobe = -1;
    auto flush = [&](bool need) {
        uint64_t m = dev::ballot(need);
        while (m) {
            const int leader = __ffsll((unsigned long long)m) - 1;
            const int l = __shfl(cur_lobe, leader, 64);
            const bool in = need && cur_lobe == l;
            m &= ~dev::ballot(in);
            const float s0 = dev::wave_sum(in ? cur0 : 0.0f);
            const float s1 = dev::wave_sum(in ? cur1 : 0.0f);
            const float s2 = dev::wave_sum(in ? cur2 : 0.0f);
            float s3 = 0.0f, s4 = 0.0f, s5 = 0.0f;
            if (l > 0) {
                s3 = dev::wave_sum(in ? cur3 : 0.0f);
                s4 = dev::wave_sum(in ? cur4 : 0.0f);
                s5 = dev::wave_sum(in ? cur5 : 0.0f);
            }
            const int r = lane - (l == 0 ? 0 : 3 + 6 * (l - 1));
            if (r >= 0 && r < (l == 0 ? 3 : 6))
                own += r == 0 ? s0 : r == 1 ? s1 : r == 2 ? s2 : r == 3 ? s3 : r == 4 ? s4 : s5;
        }
    };

    int state = kIdle;
    int lobe = 0;
    float w0 = 0.0f, w1 = 0.0f;       // weights of the Ls0 / Ls1 (or Ld) contributions
    V3 d = v3(0.0f, 0.0f, 1.0f);
    dev::RaySlab rs = dev::ray_slab(o, d, sc.box_scale);
    int32_t ref = kDone;
    int32_t* top = stack;
    dev::Hit h;
    h.leaf = -1;
    h.t = dev::kNoHit;
    h.u = h.v = 0.0f;
    int32_t best_orig = INT_MAX;
    int next_q = 0;                   // wave-uniform: next sample to hand out

    while (true) {
        // ---- fold finished rays and refill free lanes ----------------------
        // (once every sample is handed out, finished lanes keep their hits
        // and are folded together when the last ray ends)
        const uint64_t tracing = dev::ballot(state == kTracing);
        const int n_free = 64 - __popcll(tracing);
        if ((n_free >= kRefillMin && next_q < S) || tracing == 0) {
            const bool done = state == kFinished;
            flush(done && cur_lobe >= 0 && cur_lobe != lobe);
            if (done) {
                const V3 R = VOXEL ? dev::radiance_voxel(sc, h, o, d) : dev::radiance(sc, h);
                if (COUNT && h.leaf >= 0) ++n_hits;
                if (cur_lobe != lobe) {
                    cur0 = cur1 = cur2 = cur3 = cur4 = cur5 = 0.0f;
                    cur_lobe = lobe;
                }
                // diffuse: w0 = 1 and w1 = 0
                cur0 += R.x * w0;
                cur1 += R.y * w0;
                cur2 += R.z * w0;
                cur3 += R.x * w1;
                cur4 += R.y * w1;
                cur5 += R.z * w1;
                state = kIdle;
            }
            if (next_q >= S && tracing == 0) break;
            const uint64_t free_mask = ~tracing;
            if (next_q < S) {
                if (state == kIdle) {
                    const int rank = __popcll(free_mask & ((1ull << lane) - 1ull));
                    const int q = next_q + rank;
                    if (q < S) {
                        lobe = lobe_of(q, spp_d, spp_s);
                        const int s = lobe == 0 ? q : (q - spp_d) - (lobe - 1) * spp_s;
                        float xi1, xi2;
                        dev::lobe_uniforms(b.seed, rng_p, lobe, s, lobe == 0 ? b.w_d : b.w_s, xi1, xi2);
                        float sp_, cp_;
                        // azimuth 2 pi xi2: the hardware sine and cosine take the angle
                        // in turns (within 1.2e-7 of sincospif for every 24-bit xi2)
                        sp_ = __builtin_amdgcn_sinf(xi2);
                        cp_ = __builtin_amdgcn_cosf(xi2);
                        bool shoot = false;
                        if (lobe == 0) {
                            const float r = dev::sqrt_hw(xi1);
                            d = dev::to_world(ft, fb, n, r * cp_, r * sp_, dev::sqrt_hw(1.0f - xi1));
                            w0 = 1.0f;
                            w1 = 0.0f;
                            shoot = true;
                        } else {
                            const float sg = sigma[lobe - 1];
                            const float alpha = sg * sg;
                            const float a2 = alpha * alpha;
                            const float tan2 = a2 * xi1 * dev::rcp(1.0f - xi1);
                            const float cos_m = dev::rsq_ge1(1.0f + tan2);
                            const float sin_m = dev::sqrt_hw(tan2) * cos_m;
                            const V3 m = dev::to_world(ft, fb, n, sin_m * cp_, sin_m * sp_, cos_m);
                            const float om = dev::dot(wo, m);
                            if (om > 0.0f) {
                                d = (2.0f * om) * m - wo;
                                const float ci = dev::dot(n, d);
                                if (ci > 0.0f) {
                                    const float G = dev::smith_g1(a2, ci) * dev::smith_g1(a2, cos_o);
                                    const float w = G * om * dev::rcp(cos_o * cos_m);
                                    const float f = 1.0f - om;
                                    const float f2 = f * f;
                                    const float F1 = f2 * f2 * f;
                                    w0 = w * (1.0f - F1);
                                    w1 = w * F1;
                                    shoot = true;
                                }
                            }
                        }
                        if (shoot) {
                            if (COUNT) ++n_rays;
                            rs = dev::ray_slab(o, d, sc.box_scale);
                            // start below the point's chain: its siblings
                            // the ray hits are pushed level by level
                            top = stack;
                            for (int i = 0; i < chain_len; ++i) {
                                const int32_t cw = __builtin_amdgcn_readlane(chain, i);
                                if (COUNT) ++n_chain;
                                dev::chain_step(sc.nodes, cw & ~3, cw & 3, rs, top, kBlock);
                            }
                            ref = chain_end;
                            h.leaf = -1;
                            h.t = dev::kNoHit;
                            h.u = h.v = 0.0f;
                            best_orig = INT_MAX;
                            state = kTracing;
                        }
                        // an invalid specular sample counts as zero: the lane
                        // stays idle and takes another sample next time
                    }
                }
                next_q = min(S, next_q + n_free);
            }
        }
        // ---- traversal: inner nodes until every lane has parked a leaf ----
        // Lanes that are not tracing hold ref == kDone, so ref alone tells a
        // lane's position: >= 0 an inner node, other negative values a leaf.
        int32_t pend = kDone;
        const uint64_t wave = dev::ballot(true);
        while (true) {
            const bool waits = pend == kDone;
            const bool leaf = is_leaf(ref);
            // lanes without a parked leaf after this step: those that had
            // none and are not at a leaf now (taken before the branch, from
            // the two compares, so the masks stay in scalar registers)
            const uint64_t unparked = dev::ballot(waits) & ~dev::ballot(leaf);
            if (waits && leaf) {
                pend = ref;
                dev::stack_pop(ref, top, stack, kBlock);
            }
            const bool inner = ref >= 0;
            // Stop descending once fewer than kSearchMin lanes are still
            // looking for a leaf and some lane has one to test: the rest would
            // otherwise idle while the last few rays search.
            // (the masks and a 32-bit count keep the test in scalar code)
            const uint64_t searching = dev::ballot(inner) & unparked;
            const int n_searching = __builtin_popcount((uint32_t)searching) +
                                    __builtin_popcount((uint32_t)(searching >> 32));
            if (searching == 0 || (n_searching < kSearchMin && (wave & ~unparked) != 0))
                break;
            if (COUNT && lane == 0) ++n_node_steps;
            if (inner) {
                if (COUNT) ++n_nodes;
                dev::node4_step(sc.nodes, ref, top, stack, kBlock, rs, h.t);
            }
        }
        // ---- leaves ---------------------------------------------------------
        if (pend != kDone) {
            const int32_t lr = ~pend;
            const int32_t first = lr >> 3;
            const int32_t cnt = (lr & 7) + 1;
            for (int i = 0; i < cnt; ++i) {
                if (COUNT) ++n_tris;
                if (COUNT && __builtin_amdgcn_readfirstlane(lane) == lane) ++n_tri_steps;
                dev::tri_test(sc.tris, first + i, o, d, h, best_orig);
            }
        }
        if (state == kTracing && ref == kDone) state = kFinished;
    }
    // ---- flush what is left, then every owner writes its plane -----------
    flush(cur_lobe >= 0);
    if (lane < P) {
        const float cnt = lane < 3 ? (float)spp_d : (float)spp_s;
        b.out[(int64_t)slot_plane(lane, K) * os + p] = own / cnt;
    }
}

// Five wavefronts per SIMD (at most 96 VGPRs; the LDS stacks of 20 one-wave
// workgroups fit a CU's 160 KB) measured ~3 % faster than four.
#define FIPT_BAKE_OCCUPANCY __attribute__((amdgpu_waves_per_eu(5, 8)))

template <bool COUNT, bool REFILL, bool VOXEL>
__global__ __launch_bounds__(kBlock) FIPT_BAKE_OCCUPANCY void k_bake(BakeLaunch b, int32_t* counters,
                                                                     uint64_t* stats) {
    __shared__ int32_t s_stack[kStackSize * kBlock];
    const int lane = threadIdx.x & 63;
    int32_t* stack = s_stack + threadIdx.x;
    uint32_t n_rays = 0, n_nodes = 0, n_tris = 0, n_hits = 0, n_node_steps = 0, n_tri_steps = 0,
             n_chain = 0;
    const int home = (int)(blockIdx.x % kXcdCount);   // the XCD this workgroup runs on
    int tried = 0;
    for (int64_t p; (p = next_point(counters, home, tried, b.n, lane)) >= 0;) {
        if (REFILL)
            bake_point_refill<COUNT, VOXEL>(b, b.sigma, p, lane, stack, n_rays, n_nodes, n_tris, n_hits,
                                     n_node_steps, n_tri_steps, n_chain);
        else
            bake_point<COUNT, VOXEL>(b, b.sigma, p, lane, stack, n_rays, n_nodes, n_tris, n_hits);
    }
    if (COUNT) {
        // lane counters -> wave totals -> one 64-bit atomic per wave
        uint64_t v[7] = {n_rays, n_nodes, n_tris, n_hits, n_node_steps, n_tri_steps, n_chain};
        for (int k = 0; k < 7; ++k) {
            uint64_t x = v[k];
            for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
            if (lane == 0) atomicAdd((unsigned long long*)(stats + k), (unsigned long long)x);
        }
    }
}

// A job read from the tile table, its fields made wave-uniform so they stay
// in scalar registers for the whole point (read through the table, the
// compiler reloads them inside the traversal loop).  The roughness levels
// are not copied: they are read from the table by lane-varying index.
__device__ __forceinline__ BakeLaunch uniform_job(const BakeLaunch& j) {
    auto up = [](const void* v) { return (const void*)wave_uniform((int64_t)v); };
    auto u32 = [](int32_t v) { return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)v); };
    BakeLaunch b;
    b.sc.nodes = static_cast<const Bvh4Node*>(up(j.sc.nodes));
    b.sc.tris = static_cast<const TriGeom*>(up(j.sc.tris));
    b.sc.rad = static_cast<const TriRad*>(up(j.sc.rad));
    b.sc.n_tris = wave_uniform(j.sc.n_tris);
    b.sc.box_scale = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(j.sc.box_scale)));
    b.sc.vox = nullptr;   // serving scenes have no voxel cache
    b.sc.vox_res = 0;
    b.pts = static_cast<const float*>(up(j.pts));
    b.ptri = static_cast<const int32_t*>(up(j.ptri));
    b.pts_stride = wave_uniform(j.pts_stride);
    b.n = wave_uniform(j.n);
    b.p_offset = wave_uniform(j.p_offset);
    b.out = const_cast<float*>(static_cast<const float*>(up(j.out)));
    b.out_stride = wave_uniform(j.out_stride);
    b.spp_d = u32(j.spp_d);
    b.spp_s = u32(j.spp_s);
    b.w_d = (uint32_t)u32((int32_t)j.w_d);
    b.w_s = (uint32_t)u32((int32_t)j.w_s);
    b.K = u32(j.K);
    b.seed = (uint64_t)wave_uniform((int64_t)j.seed);
    b.eps = __int_as_float(u32(__float_as_int(j.eps)));
    return b;
}

// Serving: persistent bake over a list of tiles; the points of the launch
// (all tiles' points enumerated in order) are handed out as in k_bake.
__global__ __launch_bounds__(kBlock) FIPT_BAKE_OCCUPANCY void k_bake_tiles(const TileDesc* tiles,
                                                                           int32_t n_tiles,
                                                                           int32_t* counters) {
    __shared__ int32_t s_stack[kStackSize * kBlock];
    const int lane = threadIdx.x & 63;
    int32_t* stack = s_stack + threadIdx.x;
    uint32_t a = 0, bb = 0, c = 0, d = 0, e = 0, f = 0, g = 0;   // counters, unused here
    const int64_t total = tiles[n_tiles - 1].first + tiles[n_tiles - 1].job.n;
    const int home = (int)(blockIdx.x % kXcdCount);       // the XCD this workgroup runs on
    int tried = 0;
    for (int64_t p; (p = next_point(counters, home, tried, total, lane)) >= 0;) {
        // last tile whose first point is <= p
        int lo = 0, hi = n_tiles - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tiles[mid].first <= p) lo = mid;
            else hi = mid - 1;
        }
        const BakeLaunch job = uniform_job(tiles[lo].job);
        const float* sigma = tiles[lo].job.sigma;
        const int64_t q = p - tiles[lo].first;
        if (job.K <= kRefillMaxK)
            bake_point_refill<false, false>(job, sigma, q, lane, stack, a, bb, c, d, e, f, g);
        else
            bake_point<false, false>(job, sigma, q, lane, stack, a, bb, c, d);
    }
}

// One ray per thread: closest hit with the bake's traversal.
__global__ __launch_bounds__(kBlock) void k_cast_rays(DeviceScene sc, const float* rays,
                                                      int64_t n, int64_t stride, int32_t* hit_tri,
                                                      float* hit_tuv, int64_t hit_stride) {
    __shared__ int32_t s_stack[kStackSize * kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const V3 o = v3(rays[i], rays[stride + i], rays[2 * stride + i]);
    const V3 d = v3(rays[3 * stride + i], rays[4 * stride + i], rays[5 * stride + i]);
    uint32_t z0 = 0, z1 = 0;
    const dev::Hit h = dev::trace<false>(sc, o, d, s_stack + threadIdx.x, kBlock, z0, z1);
    hit_tri[i] = h.leaf >= 0 ? sc.tris[h.leaf].orig : -1;
    if (hit_tuv) {
        hit_tuv[i] = h.leaf >= 0 ? h.t : 0.0f;
        hit_tuv[hit_stride + i] = h.u;
        hit_tuv[2 * hit_stride + i] = h.v;
    }
}

// xi1, xi2 of (point p0 + i / n_samples, lobe, sample i % n_samples).
__global__ void k_lobe_uniforms(uint64_t seed, int64_t p0, int64_t total, int32_t lobe,
                                int32_t n_samples, uint32_t w, float* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    float xi1, xi2;
    dev::lobe_uniforms(seed, p0 + i / n_samples, lobe, (int)(i % n_samples), w, xi1, xi2);
    out[i] = xi1;
    out[total + i] = xi2;
}

__global__ void k_zero_counters(int32_t* counters) {
    if (threadIdx.x < kXcdCount) counters[threadIdx.x] = 0;
}

__global__ void k_set_radiance(TriRad* rad, const int32_t* order, const int32_t* tri_idx,
                               int64_t T, int kind, const float* cache, int64_t n_cache,
                               const float* emission) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T) return;
    const int32_t f = order[i];
    float c[3][3];
    for (int k = 0; k < 3; ++k) {
        const int64_t src = kind == FIPT_CACHE_VERTEX ? (int64_t)tri_idx[3 * (int64_t)f + k] : f;
        for (int ch = 0; ch < 3; ++ch) c[k][ch] = cache ? cache[ch * n_cache + src] : 0.0f;
    }
    TriRad r;
    r.c0r = c[0][0]; r.c0g = c[0][1]; r.c0b = c[0][2];
    r.c1r = c[1][0]; r.c1g = c[1][1]; r.c1b = c[1][2];
    r.c2r = c[2][0]; r.c2g = c[2][1]; r.c2b = c[2][2];
    r.ler = emission ? emission[f] : 0.0f;
    r.leg = emission ? emission[T + f] : 0.0f;
    r.leb = emission ? emission[2 * T + f] : 0.0f;
    rad[i] = r;
}

__global__ void k_set_emission(TriRad* rad, const int32_t* order, int64_t T,
                               const float* emission) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T) return;
    const int32_t f = order[i];
    rad[i].ler = emission[f];
    rad[i].leg = emission[T + f];
    rad[i].leb = emission[2 * T + f];
}

// One thread per pixel centre: camera ray -> closest hit -> shading point.
__global__ __launch_bounds__(kBlock) void k_gen_points(DeviceScene sc, CameraTable cams,
                                                       fipt_points out) {
    __shared__ int32_t s_stack[kStackSize * kBlock];
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= out.n) return;
    int c = 0;
    while (c + 1 < cams.n && p >= cams.offset[c + 1]) ++c;
    const fipt_camera cam = cams.cam[c];
    const int64_t local = p - cams.offset[c];
    const int W = cam.width, H = cam.height;
    const int i = (int)(local % W), j = (int)(local / W);
    V3 f = v3(cam.fwd[0], cam.fwd[1], cam.fwd[2]);
    f = (1.0f / sqrtf(dev::dot(f, f))) * f;
    V3 r = dev::cross(f, v3(cam.up[0], cam.up[1], cam.up[2]));
    r = (1.0f / sqrtf(dev::dot(r, r))) * r;
    const V3 u = dev::cross(r, f);
    const float th = tanf(0.5f * cam.vfov_deg * 0.017453292519943295f);
    const float aspect = (float)W / (float)H;
    const float sx = (2.0f * ((float)i + 0.5f) / (float)W - 1.0f) * th * aspect;
    const float sy = (1.0f - 2.0f * ((float)j + 0.5f) / (float)H) * th;
    V3 d = f + sx * r + sy * u;
    d = (1.0f / sqrtf(dev::dot(d, d))) * d;
    const V3 o = v3(cam.pos[0], cam.pos[1], cam.pos[2]);
    uint32_t z0 = 0, z1 = 0;
    const dev::Hit h = dev::trace<false>(sc, o, d, s_stack + threadIdx.x, kBlock, z0, z1);
    const int64_t s = out.stride;
    float* P = out.planes;
    if (h.leaf < 0) {
        for (int k = 0; k < 9; ++k) P[k * s + p] = 0.0f;
        out.tri[p] = -1;
        return;
    }
    const float4* tp = reinterpret_cast<const float4*>(sc.tris + h.leaf);
    const float4 t0 = tp[0], t1 = tp[1], t2 = tp[2];
    V3 nn = dev::cross(v3(t1.x, t1.y, t1.z), v3(t2.x, t2.y, t2.z));
    nn = (1.0f / sqrtf(dev::dot(nn, nn))) * nn;
    if (dev::dot(nn, d) > 0.0f) nn = v3(-nn.x, -nn.y, -nn.z);
    const V3 x = o + h.t * d;
    P[0 * s + p] = x.x;
    P[1 * s + p] = x.y;
    P[2 * s + p] = x.z;
    P[3 * s + p] = nn.x;
    P[4 * s + p] = nn.y;
    P[5 * s + p] = nn.z;
    P[6 * s + p] = -d.x;
    P[7 * s + p] = -d.y;
    P[8 * s + p] = -d.z;
    out.tri[p] = __float_as_int(t0.w);
}

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FIPT_EHIP, "%s launch failed: %s", what, hipGetErrorString(e));
    return FIPT_OK;
}

int device_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

}  // namespace

int launch_set_radiance(TriRad* rad, const int32_t* order, const int32_t* tri_idx, int64_t n_tris,
                        int cache_kind, const float* cache, int64_t n_cache,
                        const float* emission, void* stream) {
    const int64_t blocks = (n_tris + 255) / 256;
    hipLaunchKernelGGL(k_set_radiance, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       rad, order, tri_idx, n_tris, cache_kind, cache, n_cache, emission);
    return check_launch("set_radiance");
}

int launch_set_emission(TriRad* rad, const int32_t* order, int64_t n_tris, const float* emission,
                        void* stream) {
    const int64_t blocks = (n_tris + 255) / 256;
    hipLaunchKernelGGL(k_set_emission, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       rad, order, n_tris, emission);
    return check_launch("set_emission");
}

int launch_gen_points(const DeviceScene& sc, const CameraTable& cams, const fipt_points& out,
                      void* stream) {
    const int64_t blocks = (out.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_gen_points, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream,
                       sc, cams, out);
    return check_launch("gen_points");
}

int launch_cast_rays(const DeviceScene& sc, const float* rays, int64_t n, int64_t stride,
                     int32_t* hit_tri, float* hit_tuv, int64_t hit_stride, void* stream) {
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_cast_rays, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream,
                       sc, rays, n, stride, hit_tri, hit_tuv, hit_stride);
    return check_launch("cast_rays");
}

int launch_lobe_uniforms(uint64_t seed, int64_t p0, int64_t n_points, int32_t lobe,
                         int32_t n_samples, float* out, void* stream) {
    const int64_t total = n_points * n_samples;
    hipLaunchKernelGGL(k_lobe_uniforms, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, seed, p0, total, lobe, n_samples, stratum_width(n_samples), out);
    return check_launch("lobe_uniforms");
}

int launch_bake(const BakeLaunch& b, int32_t* counters, uint64_t* stats, void* stream) {
    // persistent grid: up to one round of resident workgroups, a multiple
    // of kXcdCount so every XCD gets the same number of workgroups
    const int64_t want = (b.n + kWaves - 1) / kWaves;
    int64_t blocks = std::min(want, (int64_t)device_cus() * kGridWavesPerCu / kWaves);
    blocks = std::max<int64_t>(kXcdCount, (blocks + kXcdCount - 1) / kXcdCount * kXcdCount);
    const dim3 grid((unsigned)blocks), block(kBlock);
    hipStream_t st = (hipStream_t)stream;
    // zeroed by a kernel, not a memset node, so a caller may capture the call
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, counters);
    const bool refill = b.K <= kRefillMaxK;
    if (b.sc.vox) {
        // radiance from the voxel cache (Sec. 4.2)
        if (stats && refill)
            hipLaunchKernelGGL((k_bake<true, true, true>), grid, block, 0, st, b, counters, stats);
        else if (stats)
            hipLaunchKernelGGL((k_bake<true, false, true>), grid, block, 0, st, b, counters, stats);
        else if (refill)
            hipLaunchKernelGGL((k_bake<false, true, true>), grid, block, 0, st, b, counters, stats);
        else
            hipLaunchKernelGGL((k_bake<false, false, true>), grid, block, 0, st, b, counters, stats);
    } else if (stats && refill)
        hipLaunchKernelGGL((k_bake<true, true, false>), grid, block, 0, st, b, counters, stats);
    else if (stats)
        hipLaunchKernelGGL((k_bake<true, false, false>), grid, block, 0, st, b, counters, stats);
    else if (refill)
        hipLaunchKernelGGL((k_bake<false, true, false>), grid, block, 0, st, b, counters, stats);
    else
        hipLaunchKernelGGL((k_bake<false, false, false>), grid, block, 0, st, b, counters, stats);
    return check_launch("bake");
}

int bake_tiles_grid_hint() { return device_cus() * kGridWavesPerCu / kWaves; }

int launch_bake_tiles(const TileDesc* tiles_dev, int32_t n_tiles, int32_t* counters_dev,
                      int32_t grid, void* stream) {
    hipLaunchKernelGGL(k_bake_tiles, dim3((unsigned)grid), dim3(kBlock), 0, (hipStream_t)stream,
                       tiles_dev, n_tiles, counters_dev);
    return check_launch("bake_tiles");
}

}  // namespace fipt
