// Internal declarations shared by the host code and the HIP kernels of
// libfipt.  Nothing here is part of the public C ABI (include/fipt.h).
#pragma once

#include <atomic>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "fipt.h"

namespace fipt {

// ---- errors ---------------------------------------------------------------
// Records a printf-style message as the calling thread's last error and
// returns `code`.
int fail(int code, const char* fmt, ...);
void clear_error();

// ---- BVH layout -----------------------------------------------------------
// Binary BVH.  A node holds the boxes of both children so one 64-byte fetch
// decides which children a ray enters.  Child reference: >= 0 -> internal
// node index; < 0 -> leaf ~((first << 3) | (count - 1)), first = position of
// its first triangle in leaf order, count in [1, 8].
constexpr int kLeafMax = 8;
constexpr int kStackSize = 32;     // LDS traversal stack entries per lane
constexpr int kMaxInnerDepth = 30; // deepest internal node (root = 0)

struct alignas(16) BvhNode {
    float c0lx, c0hx, c0ly, c0hy;  // child 0 box, x and y
    float c1lx, c1hx, c1ly, c1hy;  // child 1 box, x and y
    float c0lz, c0hz, c1lz, c1hz;  // both boxes, z
    int32_t child0, child1, pad0, pad1;
};
static_assert(sizeof(BvhNode) == 64, "node is one 64-byte fetch");

// Triangle in leaf order: first vertex, the two edges from it, and the
// original triangle index (for ties and for reporting).  48 bytes.
struct alignas(16) TriGeom {
    float v0x, v0y, v0z;
    int32_t orig;
    float e1x, e1y, e1z, pad1;
    float e2x, e2y, e2z, pad2;
};
static_assert(sizeof(TriGeom) == 48, "triangle is three 16-byte fetches");

// Radiance record in leaf order: cache value at the three corners (equal
// for a per-triangle cache) and the triangle's emission.  48 bytes.
struct alignas(16) TriRad {
    float c0r, c0g, c0b, c1r;
    float c1g, c1b, c2r, c2g;
    float c2b, ler, leg, leb;
};
static_assert(sizeof(TriRad) == 48, "radiance record is three 16-byte fetches");

inline int32_t leaf_ref(int64_t first, int count) {
    return ~static_cast<int32_t>((first << 3) | (count - 1));
}

// 4-wide BVH collapsed from the binary one.  The collapse works on Wide4
// nodes: the single-precision boxes of up to four children (structure of
// arrays) and their references (same encoding as the binary tree;
// kEmptyChild marks an unused slot).  It keeps the stack pushes along every
// root-to-leaf path within kStackSize, so the traversal stack cannot
// overflow.
constexpr int32_t kEmptyChild = -2147483647;   // INT32_MIN + 1: never a leaf reference
struct Wide4 {
    float lo[3][4], hi[3][4];   // [axis][slot]
    int32_t child[4];
};

// The device form of a 4-wide node, 128 bytes of which the traversal reads
// the first 80 in five 16-byte loads.  Bounds are in units of 2^E, one
// exponent E for the whole tree (HostBvh::box_exp).  Per axis, q[axis]
// holds the slots' low bounds then high bounds as signed half-precision
// offsets from org[axis]:  bound = (org + offset) 2^E.  The origin is the
// low bound of the slot thinnest on that axis, so a flat box (a wall, a
// floor) keeps its thickness and a ray leaving such a surface does not
// start inside it; other bounds carry the half-precision error of their
// distance from the origin.  Offsets are rounded outward (lows down, highs
// up), so every decoded box contains the single-precision box it encodes;
// an unused slot has low +inf and high -inf, which no ray enters.
struct alignas(16) Bvh4Node {
    uint16_t q[3][8];    // bytes 0..47: x, y, z; each lo[0..3], hi[0..3]
    float org[3];        // bytes 48..59
    int32_t spare;       // bytes 60..63
    int32_t child[4];    // bytes 64..79: an inner child as the byte offset of its
                         // node (index x 128), a leaf as in the binary tree
    int32_t pad[12];
};
static_assert(sizeof(Bvh4Node) == 128, "4-wide node is one 128-byte line");
// node byte offsets stay below 2^31: an inner reference is a non-negative
// int32 and its low seven bits are zero
constexpr int64_t kMaxNodes4 = int64_t(1) << 24;
inline int32_t node4_ref(int32_t child) {
    return child >= 0 ? (int32_t)((uint32_t)child << 7) : child;
}

struct HostBvh {
    std::vector<BvhNode> nodes;
    std::vector<Wide4> wide4;      // the collapse, single precision
    std::vector<Bvh4Node> nodes4;  // its device encoding
    std::vector<TriGeom> tris;     // leaf order
    std::vector<int32_t> order;    // leaf position -> original triangle
    int max_depth = 0;
    int max_push4 = 0;             // most stack pushes on a path of the 4-wide tree
    int box_exp = 0;               // nodes4 bounds are in units of 2^box_exp
    float bmin[3] = {0, 0, 0}, bmax[3] = {0, 0, 0};
};

// Binned-SAH top-down build; deterministic; internal depth capped at
// kMaxInnerDepth by switching to object-median splits when needed.
int build_bvh(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
              HostBvh* out);

// ---- kernels (launchers defined in the .hip files) -------------------------
// Width of each of n equal segments of the 32-bit line, floor(2^32 / n);
// 0 stands for 2^32 (n = 1).
inline uint32_t stratum_width(int64_t n) {
    return n <= 1 ? 0u : (uint32_t)((uint64_t(1) << 32) / (uint64_t)n);
}

struct DeviceScene {
    const Bvh4Node* nodes;
    const TriGeom* tris;
    const TriRad* rad;
    int64_t n_tris;
    float box_scale;   // 2^E: the unit of the node bounds
    // Voxel radiance cache (NULL unless the scene uses one), stored sparse in
    // bricks of 4 x 4 x 4 voxels: voxel (i, j, k) belongs to brick
    // (i / 4, j / 4, k / 4), numbered (bz B + by) B + bx with B = ceil(R / 4),
    // as bit ((k % 4) * 4 + j % 4) * 4 + i % 4 of that brick's word
    // {mask low, mask high, occupied voxels in earlier bricks, 0}; an
    // occupied voxel's value (rgb, w unused) is vox[rank + occupied voxels
    // before it in its brick], an empty one is zero.  A point x lies in
    // voxel floor((x - vox_lo) * vox_scale), clamped to [0, R - 1].
    const uint4* vox_words;
    const float4* vox;
    int32_t vox_res;
    int32_t vox_bricks;   // B
    float vox_lo[3];
    float vox_scale[3];   // R / (hi - lo) per axis
};

int launch_set_radiance(TriRad* rad, const int32_t* order, const int32_t* tri_idx,
                        int64_t n_tris, int cache_kind, const float* cache, int64_t n_cache,
                        const float* emission, void* stream);
int launch_set_emission(TriRad* rad, const int32_t* order, int64_t n_tris,
                        const float* emission, void* stream);
// Voxel cache planes [3][stride] of an R^3 grid -> the scene's sparse brick
// form: occupancy words with ranks (and the occupied count in *total), then
// the occupied values.
int launch_voxel_words(uint4* words, const float* cache, int64_t stride, int32_t res,
                       uint32_t* tile_sum, int64_t* total, void* stream);
constexpr int64_t kVoxelScanTile = 1024;   // words per scan tile
int launch_voxel_compact(float4* dst, const uint4* words, const float* cache, int64_t stride,
                         int32_t res, void* stream);
constexpr int32_t kMaxVoxelRes = 512;
// Cameras travel by value in the kernel arguments (no staging allocation).
constexpr int kMaxCameras = 48;
struct CameraTable {
    fipt_camera cam[kMaxCameras];
    int64_t offset[kMaxCameras + 1];  // first point of each camera
    int32_t n;
};
int launch_gen_points(const DeviceScene& sc, const CameraTable& cams, const fipt_points& out,
                      void* stream);
int launch_cast_rays(const DeviceScene& sc, const float* rays, int64_t n, int64_t stride,
                     int32_t* hit_tri, float* hit_tuv, int64_t hit_stride, void* stream);
int launch_lobe_uniforms(uint64_t seed, int64_t p0, int64_t n_points, int32_t lobe,
                         int32_t n_samples, float* out, void* stream);

struct BakeLaunch {
    DeviceScene sc;
    const float* pts;
    const int32_t* ptri;
    int64_t pts_stride;
    int64_t n;            // points
    int64_t p_offset;     // added to the point index for the RNG counter
    float* out;
    int64_t out_stride;
    int32_t spp_d, spp_s, K;
    uint32_t w_d, w_s;    // stratum widths stratum_width(spp_d), stratum_width(spp_s)
    float sigma[FIPT_MAX_LEVELS];
    uint64_t seed;
    float eps;
};
// counters_dev: kXcdCount int32 point counters owned by this launch; the
// launcher zeroes them on `stream` before the kernel.
int launch_bake(const BakeLaunch& b, int32_t* counters_dev, uint64_t* stats, void* stream);

// Stage-3 refinement (fipt_refine): the material grid, the path rules and
// the scene's emitter list (leaf positions, count on the device).
struct RefineLaunch {
    const float* grid;    // [5][res^3]
    int32_t res;
    float bmin[3], bmax[3];
    float sigma_diffuse;
    int32_t max_vertices;
    int32_t flags;
    const int32_t* emit;
    const int32_t* n_emit;
};
// Emitters (some channel of emission > 0) in ascending original index into
// list (leaf positions) and their number into *count; blocks: one int32 per
// 256 triangles of scratch.
int launch_emitter_list(const TriRad* rad, const int32_t* leaf_of, int64_t n_tris, int32_t* blocks,
                        int32_t* list, int32_t* count, void* stream);
int launch_refine(const BakeLaunch& b, const RefineLaunch& r, int32_t* counters, void* stream);

// MI355X has 8 XCDs (dies, each with its own L2); the dispatcher places
// workgroup i of a launch on XCD i % kXcdCount.
constexpr int kXcdCount = 8;

// Serving: a tile is a contiguous run of one request's points.
struct TileDesc {
    BakeLaunch job;       // job.n = points in the tile, pointers already offset
    int64_t first;        // points of all earlier tiles in the launch
};
// counters_dev: kXcdCount zeroed int32 counters.
int launch_bake_tiles(const TileDesc* tiles_dev, int32_t n_tiles, int32_t* counters_dev,
                      int32_t grid, void* stream);
int bake_tiles_grid_hint();

// Terms of the masked loss (Eq. 12 / 15 with the prior of Eq. 17); a NULL
// RenderLossMask* selects the plain loss.
struct RenderLossMask {
    const float* alpha;  // [n] or NULL (zero)
    float* grad_alpha;   // [n] or NULL
    double lambda_d;
};
// `partials` receives one double per workgroup (render_loss_partials(n)
// of them) before the final sum writes loss[0].
int launch_render_loss(const float* sh, int64_t sh_stride, int64_t n, int32_t K,
                       const float* sigma_host, const float* mat, int64_t mat_stride,
                       const float* obs, int64_t obs_stride, int32_t tone, double* loss,
                       double* partials, float* grad, int64_t grad_stride, float* Lr,
                       int64_t lr_stride, const RenderLossMask* mask, void* stream);
// Workgroups (= partial sums) of the render-loss launch for n points.
int render_loss_partials(int64_t n);
// Device address of the library's static partials array on the current
// device, and its capacity in doubles.
int render_loss_scratch(double** out, int64_t* capacity);
int launch_scale_by(const float* x, int64_t n, const double* f, float* out, void* stream);
// Bandwidth probe: kind 0 copy c = a, kind 1 triad c = a + s b.
int launch_stream(int32_t kind, const float* a, const float* b, float* c, int64_t n, float s,
                  void* stream);
int launch_grid_gather(const float* grid, int32_t C, int32_t R, const float* bmin,
                       const float* bmax, const float* pos, int64_t pos_stride, int64_t n,
                       float* out, int64_t out_stride, void* stream);

// The grid adjoint works on node bricks of kBrickX x kBrickY x kBrickZ
// nodes.  A point's home brick holds the lower corner of its cell; its points
// are cut into columns of at most kColumnMax points of one cell, and a brick
// lists its home columns and the columns of the lower neighbours' cells whose
// upper corners are its nodes (halo columns).  A brick's column list is cut
// into work units of at most kAdjUnit columns, one workgroup each; a brick of
// several units has its units' node sums combined in unit order.
constexpr int kBrickX = 8, kBrickY = 8, kBrickZ = 8;
constexpr int kBrickNodes = kBrickX * kBrickY * kBrickZ;
#ifndef FIPT_COLUMN_MAX
#define FIPT_COLUMN_MAX 8
#endif
constexpr int kColumnMax = FIPT_COLUMN_MAX;
#ifndef FIPT_ADJ_UNIT
#define FIPT_ADJ_UNIT 256
#endif
constexpr int kAdjUnit = FIPT_ADJ_UNIT;

struct GridPlanDev {
    int32_t res;
    int64_t n_points;
    float bmin[3], bmax[3];
    int32_t nb[3];          // bricks per axis, ceil(res / brick extent)
    int64_t n_bricks;
    float4* pts;            // [n_points] (x, y, z, point index as int bits), by (home brick, cell, index)
    int2* cols;             // [n_cols] (first point in pts, count | (lx+1) << 5 | (ly+1) << 11 | (lz+1) << 17),
                            // (lx, ly, lz) the cell's position relative to the brick's first node, >= -1
    int64_t n_cols;
    int4* units;            // [n_units] (brick, first column, end column, scratch slot or -1 when the
                            // unit is its brick's only one), every brick at least once, most columns first
    int64_t n_units;
    int4* multi;            // [n_multi] (brick, first scratch slot, unit count, 0): bricks of several units
    int64_t n_multi;
    double* part;           // [n_slots][8][kBrickNodes] node sums of the units of those bricks
    int64_t n_slots;
    int32_t* hcol;          // [n_cols] home column (numbered in point order) of each column entry
    int32_t* colq;          // [n_points] home column of each point in sorted order
    int64_t n_home;         // home columns: each cell's run of points cut into columns
    float* csum;            // [n_home][40] column sums of the fused loss: channel ch, corner c at
                            // ch * 8 + c (160-byte records)
};
int launch_grid_scatter(const GridPlanDev& p, const float* gp, int32_t C, int64_t gp_stride,
                        float* grad_grid, void* stream);
// Fused material fetch + render + loss + adjoint over a plan's points given
// in the plan's order; per-point gradients also go to gq[5][gqs] when gq is
// not NULL.
int launch_grid_render_loss(const GridPlanDev& p, const float* grid, const float* sh, int64_t ss,
                            int32_t K, const float* sigma, const float* obs, int64_t os,
                            int32_t tone, double* loss, double* partials, float* gq, int64_t gqs,
                            float* grad_grid, void* stream);
int launch_plan_permute(const GridPlanDev& p, const float* src, int32_t planes, int64_t ss,
                        float* dst, int64_t ds, void* stream);

}  // namespace fipt

// Work-counter slots of a scene's bakes: each fipt_bake call takes the next
// slot and first makes its stream wait for the slot's previous launch, so
// no two launches in flight share counters, on any streams.
constexpr int kBakeSlots = 16;

struct fipt_scene_s {
    int32_t device = 0;
    int64_t n_tris = 0, n_verts = 0, n_nodes = 0;
    int32_t max_depth = 0;
    int32_t cache_kind = -1;
    float box_scale = 1.0f;        // 2^E of the node bounds
    float bmin[3] = {0, 0, 0}, bmax[3] = {0, 0, 0};
    fipt::Bvh4Node* d_nodes = nullptr;   // 4-wide nodes
    fipt::TriGeom* d_tris = nullptr;
    fipt::TriRad* d_rad = nullptr;
    uint4* d_vox_words = nullptr;  // voxel occupancy words, when cache_kind is FIPT_CACHE_VOXEL
    int64_t vox_word_capacity = 0;
    float4* d_vox = nullptr;       // occupied voxels' values
    int64_t vox_capacity = 0;      // values allocated
    int64_t* d_vox_total = nullptr;  // occupied count, read back by the set-up call
    uint32_t* d_vox_tiles = nullptr; // per scan tile of words: its total, then its offset
    int32_t vox_res = 0;
    float vox_lo[3] = {0, 0, 0}, vox_scale[3] = {0, 0, 0};
    int32_t* d_order = nullptr;    // leaf position -> original triangle
    int32_t* d_leaf_of = nullptr;  // original triangle -> leaf position
    int32_t* d_emit = nullptr;     // [T + 1] emitters' leaf positions (refinement), count last
    int32_t* d_emit_blocks = nullptr;  // [ceil(T / 256)] scan scratch of the emitter list
    hipEvent_t refine_done = nullptr;  // last refinement's completion (it rewrites d_emit)
    std::mutex refine_mu;
    int32_t* d_tri_idx = nullptr;  // original [T][3] vertex indices
    int32_t* d_counters = nullptr;  // [kBakeSlots][kXcdCount]
    hipEvent_t slot_done[kBakeSlots] = {};
    int next_slot = 0;
    std::mutex slot_mu;
    int64_t bytes = 0;
    std::atomic<int> refs{0};      // serving requests referencing the scene
    fipt::DeviceScene view() const {
        const bool vox = cache_kind == FIPT_CACHE_VOXEL;
        return {d_nodes, d_tris, d_rad, n_tris, box_scale, vox ? d_vox_words : nullptr,
                vox ? d_vox : nullptr, vox ? vox_res : 0, vox ? (vox_res + 3) / 4 : 0,
                {vox_lo[0], vox_lo[1], vox_lo[2]}, {vox_scale[0], vox_scale[1], vox_scale[2]}};
    }
};
