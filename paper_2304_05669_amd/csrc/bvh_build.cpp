// Host construction of the binary BVH the bake traverses.
//
// Top-down binned surface-area-heuristic build (32 bins per axis over the
// triangle centroids), single-threaded and therefore deterministic.  Child
// boxes are widened outward by a few units in the last place so that the
// single-precision slab test on the GPU never rejects a box a ray actually
// touches (flat, axis-aligned walls give boxes of zero thickness).
//
// The depth of internal nodes is capped at kMaxInnerDepth: when the
// remaining budget would not suffice for a subtree built by halving, the
// build switches to object-median splits, which need ceil(log2(n / 8))
// further levels.  The traversal's fixed LDS stack (kStackSize entries per
// lane) therefore can never overflow.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "fipt_internal.hpp"

namespace fipt {
namespace {

struct Box {
    float lo[3], hi[3];
    void reset() {
        for (int k = 0; k < 3; ++k) {
            lo[k] = INFINITY;
            hi[k] = -INFINITY;
        }
    }
    void grow(const Box& b) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], b.lo[k]);
            hi[k] = std::max(hi[k], b.hi[k]);
        }
    }
    void grow(const float* p) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], p[k]);
            hi[k] = std::max(hi[k], p[k]);
        }
    }
    double area() const {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = std::max(0.0, (double)hi[k] - (double)lo[k]);
        return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
    }
};

struct Prim {
    Box b;
    float c[3];
    int32_t id;
};

constexpr int kBins = 32;

int ceil_log2(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

// 2^-20 relative, plus the smallest normal float so a bound at exactly zero
// still moves (an absolute floor any larger would inflate the boxes of a
// scene whose coordinates are themselves that small)
float widen_lo(float v) {
    float e = std::fabs(v) * 9.5367431640625e-07f + 1.17549435e-38f;
    return v - e;
}
float widen_hi(float v) {
    float e = std::fabs(v) * 9.5367431640625e-07f + 1.17549435e-38f;
    return v + e;
}

class Builder {
  public:
    Builder(const float* verts, const int32_t* tris, int64_t n_tris, HostBvh* out)
        : verts_(verts), tris_(tris), out_(out) {
        prims_.resize(n_tris);
        for (int64_t f = 0; f < n_tris; ++f) {
            Prim& p = prims_[f];
            p.b.reset();
            for (int k = 0; k < 3; ++k) p.b.grow(verts + 3 * (int64_t)tris[3 * f + k]);
            for (int k = 0; k < 3; ++k) p.c[k] = 0.5f * (p.b.lo[k] + p.b.hi[k]);
            p.id = (int32_t)f;
        }
    }

    void run() {
        out_->nodes.clear();
        out_->tris.clear();
        out_->order.clear();
        out_->nodes.reserve(prims_.size() / 2 + 2);
        out_->tris.reserve(prims_.size());
        out_->order.reserve(prims_.size());
        max_depth_ = 0;
        Box root_box = bounds(0, (int64_t)prims_.size());
        // The root is always an internal node (traversal starts by fetching
        // node 0).  A one-triangle scene references its leaf from both
        // children.
        int64_t n = (int64_t)prims_.size();
        int64_t root = alloc_node();
        if (n == 1) {
            int32_t leaf = make_leaf(0, 1);
            set_child(root, 0, leaf, root_box);
            set_child(root, 1, leaf, root_box);
        } else {
            split_into(root, 0, n, root_box, 0);
        }
        out_->max_depth = max_depth_;
        for (int k = 0; k < 3; ++k) {
            out_->bmin[k] = root_box.lo[k];
            out_->bmax[k] = root_box.hi[k];
        }
    }

  private:
    const float* verts_;
    const int32_t* tris_;
    HostBvh* out_;
    std::vector<Prim> prims_;
    int max_depth_ = 0;

    Box bounds(int64_t b, int64_t e) const {
        Box box;
        box.reset();
        for (int64_t i = b; i < e; ++i) box.grow(prims_[i].b);
        return box;
    }

    int64_t alloc_node() {
        out_->nodes.push_back(BvhNode{});
        return (int64_t)out_->nodes.size() - 1;
    }

    int32_t make_leaf(int64_t b, int64_t e) {
        int64_t first = (int64_t)out_->tris.size();
        for (int64_t i = b; i < e; ++i) {
            int32_t f = prims_[i].id;
            const float* p0 = verts_ + 3 * (int64_t)tris_[3 * (int64_t)f + 0];
            const float* p1 = verts_ + 3 * (int64_t)tris_[3 * (int64_t)f + 1];
            const float* p2 = verts_ + 3 * (int64_t)tris_[3 * (int64_t)f + 2];
            TriGeom t;
            t.v0x = p0[0];
            t.v0y = p0[1];
            t.v0z = p0[2];
            t.orig = f;
            t.e1x = p1[0] - p0[0];
            t.e1y = p1[1] - p0[1];
            t.e1z = p1[2] - p0[2];
            t.pad1 = 0.0f;
            t.e2x = p2[0] - p0[0];
            t.e2y = p2[1] - p0[1];
            t.e2z = p2[2] - p0[2];
            t.pad2 = 0.0f;
            out_->tris.push_back(t);
            out_->order.push_back(f);
        }
        return leaf_ref(first, (int)(e - b));
    }

    void set_child_raw(int64_t node, int which, int32_t ref, const Box& bx) {
        BvhNode& nd = out_->nodes[node];
        if (which == 0) {
            nd.c0lx = bx.lo[0]; nd.c0hx = bx.hi[0];
            nd.c0ly = bx.lo[1]; nd.c0hy = bx.hi[1];
            nd.c0lz = bx.lo[2]; nd.c0hz = bx.hi[2];
            nd.child0 = ref;
        } else {
            nd.c1lx = bx.lo[0]; nd.c1hx = bx.hi[0];
            nd.c1ly = bx.lo[1]; nd.c1hy = bx.hi[1];
            nd.c1lz = bx.lo[2]; nd.c1hz = bx.hi[2];
            nd.child1 = ref;
        }
        nd.pad0 = nd.pad1 = 0;
    }

    void set_child(int64_t node, int which, int32_t ref, const Box& b) {
        Box w;
        for (int k = 0; k < 3; ++k) {
            w.lo[k] = widen_lo(b.lo[k]);
            w.hi[k] = widen_hi(b.hi[k]);
        }
        set_child_raw(node, which, ref, w);
    }

    // Choose a split of [b, e) (n > 1); returns the partition point.
    int64_t choose_split(int64_t b, int64_t e, const Box& box, int depth, bool* leaf_ok) {
        int64_t n = e - b;
        Box cb;
        cb.reset();
        for (int64_t i = b; i < e; ++i) cb.grow(prims_[i].c);
        int need = ceil_log2((n + kLeafMax - 1) / kLeafMax);
        bool force_median = depth + need >= kMaxInnerDepth - 1;
        int axis = 0;
        float ext = cb.hi[0] - cb.lo[0];
        for (int k = 1; k < 3; ++k)
            if (cb.hi[k] - cb.lo[k] > ext) {
                ext = cb.hi[k] - cb.lo[k];
                axis = k;
            }
        *leaf_ok = false;
        if (n <= kLeafMax && (force_median || !(ext > 0.0f))) {
            // out of depth budget, or nothing to separate: a leaf
            *leaf_ok = true;
            return b + n / 2;
        }
        if (!(ext > 0.0f)) {
            // all centroids coincide: split by index
            return b + n / 2;
        }
        if (force_median) return median_split(b, e, axis);

        // binned SAH over all three axes
        double best_cost = INFINITY;
        int best_axis = -1, best_bin = -1;
        for (int a = 0; a < 3; ++a) {
            float lo = cb.lo[a], hi = cb.hi[a];
            if (!(hi > lo)) continue;
            float scale = kBins / (hi - lo);
            Box bb[kBins];
            int64_t cnt[kBins];
            for (int i = 0; i < kBins; ++i) {
                bb[i].reset();
                cnt[i] = 0;
            }
            for (int64_t i = b; i < e; ++i) {
                int k = (int)((prims_[i].c[a] - lo) * scale);
                k = std::min(std::max(k, 0), kBins - 1);
                bb[k].grow(prims_[i].b);
                ++cnt[k];
            }
            double right_area[kBins];
            int64_t right_cnt[kBins];
            Box acc;
            acc.reset();
            int64_t c = 0;
            for (int i = kBins - 1; i > 0; --i) {
                acc.grow(bb[i]);
                c += cnt[i];
                right_area[i] = acc.area();
                right_cnt[i] = c;
            }
            acc.reset();
            c = 0;
            for (int i = 0; i < kBins - 1; ++i) {
                acc.grow(bb[i]);
                c += cnt[i];
                if (c == 0 || right_cnt[i + 1] == 0) continue;
                double cost = acc.area() * (double)c + right_area[i + 1] * (double)right_cnt[i + 1];
                if (cost < best_cost) {
                    best_cost = cost;
                    best_axis = a;
                    best_bin = i;
                }
            }
        }
        double parent = box.area();
        // SAH with traversal cost 1 and intersection cost 1 per triangle
        double split_cost = 1.0 + (parent > 0 ? best_cost / parent : INFINITY);
        double leaf_cost = (double)n;
        if (n <= kLeafMax && leaf_cost <= split_cost) *leaf_ok = true;
        if (best_axis < 0) return median_split(b, e, axis);
        float lo = cb.lo[best_axis];
        float scale = kBins / (cb.hi[best_axis] - lo);
        auto mid = std::stable_partition(prims_.begin() + b, prims_.begin() + e,
                                         [&](const Prim& p) {
                                             int k = (int)((p.c[best_axis] - lo) * scale);
                                             k = std::min(std::max(k, 0), kBins - 1);
                                             return k <= best_bin;
                                         });
        int64_t m = mid - prims_.begin();
        if (m == b || m == e) return median_split(b, e, axis);
        return m;
    }

    int64_t median_split(int64_t b, int64_t e, int axis) {
        int64_t m = b + (e - b) / 2;
        std::nth_element(prims_.begin() + b, prims_.begin() + m, prims_.begin() + e,
                         [axis](const Prim& x, const Prim& y) {
                             if (x.c[axis] != y.c[axis]) return x.c[axis] < y.c[axis];
                             return x.id < y.id;
                         });
        return m;
    }

    // Build the subtree over [b, e) and return its child reference.
    int32_t build(int64_t b, int64_t e, const Box& box, int depth) {
        int64_t n = e - b;
        if (n <= kLeafMax) {
            if (n == 1) return make_leaf(b, e);
            bool leaf_ok = false;
            // leaf test needs the split cost; reuse choose_split without
            // committing when a leaf wins (partition order does not matter
            // for a leaf).
            int64_t m = choose_split(b, e, box, depth, &leaf_ok);
            if (leaf_ok) return make_leaf(b, e);
            int64_t node = alloc_node();
            finish_node(node, b, m, e, depth);
            return (int32_t)node;
        }
        int64_t node = alloc_node();
        split_into(node, b, e, box, depth);
        return (int32_t)node;
    }

    void split_into(int64_t node, int64_t b, int64_t e, const Box& box, int depth) {
        bool leaf_ok = false;
        int64_t m = choose_split(b, e, box, depth, &leaf_ok);
        finish_node(node, b, m, e, depth);
    }

    void finish_node(int64_t node, int64_t b, int64_t m, int64_t e, int depth) {
        max_depth_ = std::max(max_depth_, depth);
        Box lb = bounds(b, m), rb = bounds(m, e);
        int32_t l = build(b, m, lb, depth + 1);
        int32_t r = build(m, e, rb, depth + 1);
        set_child(node, 0, l, lb);
        set_child(node, 1, r, rb);
    }
};

// Collapse of the binary tree into 4-wide nodes.  A 4-wide node takes the
// two children of a binary node and repeatedly replaces the internal child
// of largest surface area by its own two children, up to four.  A node with
// c children pushes at most c - 1 stack entries, so an expansion is taken
// only if the pushes of this node plus the binary depth of every child
// (what that child costs if nothing below it is collapsed) stay within the
// remaining budget; the root's budget is the stack size.
class Collapser {
  public:
    explicit Collapser(HostBvh* b) : b_(b) {
        const int64_t n = (int64_t)b->nodes.size();
        need_.assign(n, 0);
        // children follow their parent in depth-first order
        for (int64_t i = n - 1; i >= 0; --i) {
            const BvhNode& nd = b->nodes[i];
            need_[i] = 1 + std::max(need(nd.child0), need(nd.child1));
        }
    }

    void run() {
        b_->wide4.clear();
        b_->wide4.reserve(b_->nodes.size() / 2 + 1);
        max_push_ = 0;
        collapse(0, kStackSize, 0);
        b_->max_push4 = max_push_;
    }

  private:
    struct Child {
        int32_t ref;
        float lo[3], hi[3];
    };
    HostBvh* b_;
    std::vector<int> need_;
    int max_push_ = 0;

    int need(int32_t ref) const { return ref >= 0 ? need_[ref] : 0; }

    static double area(const Child& c) {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = std::max(0.0, (double)c.hi[k] - (double)c.lo[k]);
        return d[0] * d[1] + d[1] * d[2] + d[2] * d[0];
    }

    void children_of(int32_t ref, Child out[2]) const {
        const BvhNode& nd = b_->nodes[ref];
        out[0] = {nd.child0, {nd.c0lx, nd.c0ly, nd.c0lz}, {nd.c0hx, nd.c0hy, nd.c0hz}};
        out[1] = {nd.child1, {nd.c1lx, nd.c1ly, nd.c1lz}, {nd.c1hx, nd.c1hy, nd.c1hz}};
    }

    int cost(const std::vector<Child>& c) const {
        int m = 0;
        for (const Child& x : c) m = std::max(m, need(x.ref));
        return (int)c.size() - 1 + m;
    }

    int32_t collapse(int32_t ref, int budget, int pushed) {
        if (ref < 0) {
            max_push_ = std::max(max_push_, pushed);
            return ref;
        }
        Child two[2];
        children_of(ref, two);
        std::vector<Child> c(two, two + 2);
        while (c.size() < 4) {
            std::vector<int> order;
            for (int i = 0; i < (int)c.size(); ++i)
                if (c[i].ref >= 0) order.push_back(i);
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int b) { return area(c[a]) > area(c[b]); });
            bool expanded = false;
            for (int i : order) {
                std::vector<Child> trial;
                for (int j = 0; j < (int)c.size(); ++j)
                    if (j != i) trial.push_back(c[j]);
                Child g[2];
                children_of(c[i].ref, g);
                trial.insert(trial.begin() + i, g, g + 2);
                if (cost(trial) <= budget) {
                    c = trial;
                    expanded = true;
                    break;
                }
            }
            if (!expanded) break;
        }
        const int32_t idx = (int32_t)b_->wide4.size();
        b_->wide4.push_back(Wide4{});
        const int pushes = (int)c.size() - 1;
        int32_t refs[4];
        for (int i = 0; i < (int)c.size(); ++i)
            refs[i] = collapse(c[i].ref, budget - pushes, pushed + pushes);
        Wide4& nd = b_->wide4[idx];
        for (int i = 0; i < 4; ++i) {
            if (i < (int)c.size()) {
                for (int k = 0; k < 3; ++k) {
                    nd.lo[k][i] = c[i].lo[k];
                    nd.hi[k][i] = c[i].hi[k];
                }
                nd.child[i] = refs[i];
            } else {
                for (int k = 0; k < 3; ++k) {
                    nd.lo[k][i] = INFINITY;
                    nd.hi[k][i] = -INFINITY;
                }
                nd.child[i] = kEmptyChild;
            }
        }
        return idx;
    }
};


// Surface-area-guided collapse of the binary tree into 4-wide nodes, by
// dynamic programming over the binary tree (the scheme of Ylitie et al.,
// HPG 2017, for 8-wide trees, here with 4 slots).  For a binary node x let
// C(x) be the least expected cost of x as a 4-wide node of its own and
// D(x, j) the least expected cost of covering x's subtree with at most j
// children of the 4-wide node above it:
//   C(x)    = A(x) c_node + min over k of D(l, k) + D(r, 4 - k)
//   D(x, 1) = C(x)
//   D(x, j) = min(D(x, j - 1), min over k of D(l, k) + D(r, j - k))
// where l, r are x's children, a leaf costs A(leaf) c_tri n_tris in any
// number of slots, and A is a box's surface area (proportional to the
// chance that a ray enters it).  c_node is the cost of one 4-wide node step
// and c_tri that of one triangle test, in the same unit.
//
// The unconstrained optimum can push more entries on a path than the
// traversal stack holds, so the tree is built top-down under a push budget:
// at each 4-wide node, among the ways of covering its two children with 2,
// 3 or 4 slots (each slot's subtree taken as the table prescribes), the
// cheapest is chosen whose slots can still be built within the remaining
// budget at one push per binary level (their binary depth).  Covering the
// two children themselves always qualifies, so the build never fails, and
// no path pushes more than kStackSize entries.
class OptimalCollapser {
  public:
    static constexpr double kNodeCost = 1.0;
    static constexpr double kTriCost = 0.4;

    explicit OptimalCollapser(HostBvh* b) : b_(b) {}

    void run() {
        const int64_t n = (int64_t)b_->nodes.size();
        C_.assign(n, 0.0);
        D_.assign(n, {0.0, 0.0, 0.0, 0.0, 0.0});
        how_.assign(n, {0, 0, 0, 0, 0});
        need_.assign(n, 0);
        // children follow their parent in depth-first order
        for (int64_t i = n - 1; i >= 0; --i) solve((int32_t)i);
        b_->wide4.clear();
        b_->wide4.reserve(n / 2 + 1);
        max_push_ = 0;
        build(0, kStackSize, 0);
        b_->max_push4 = max_push_;
    }

  private:
    struct Slot {
        int32_t ref;
        float lo[3], hi[3];
    };
    HostBvh* b_;
    std::vector<double> C_;
    std::vector<std::array<double, 5>> D_;   // index j = 1..4
    std::vector<std::array<int, 5>> how_;    // D: 0 itself, -1 fewer slots, k split
    std::vector<int> need_;                  // binary depth: pushes with 2-wide nodes only
    int max_push_ = 0;

    static double area(const float* lo, const float* hi) {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = std::max(0.0, (double)hi[k] - (double)lo[k]);
        return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
    }
    Slot slot(int32_t node, int which) const {
        const BvhNode& nd = b_->nodes[node];
        if (which == 0) return {nd.child0, {nd.c0lx, nd.c0ly, nd.c0lz}, {nd.c0hx, nd.c0hy, nd.c0hz}};
        return {nd.child1, {nd.c1lx, nd.c1ly, nd.c1lz}, {nd.c1hx, nd.c1hy, nd.c1hz}};
    }
    double cost(const Slot& s, int j) const {
        if (s.ref >= 0) return D_[s.ref][j];
        const int count = ((~s.ref) & 7) + 1;
        return area(s.lo, s.hi) * kTriCost * count;
    }
    int need(const Slot& s) const { return s.ref >= 0 ? need_[s.ref] : 0; }
    void solve(int32_t x) {
        const Slot l = slot(x, 0), r = slot(x, 1);
        need_[x] = 1 + std::max(need(l), need(r));
        float lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(l.lo[k], r.lo[k]);
            hi[k] = std::max(l.hi[k], r.hi[k]);
        }
        double best = INFINITY;
        for (int k = 1; k <= 3; ++k) best = std::min(best, cost(l, k) + cost(r, 4 - k));
        C_[x] = area(lo, hi) * kNodeCost + best;
        D_[x][1] = C_[x];
        how_[x][1] = 0;
        for (int j = 2; j <= 4; ++j) {
            double d = D_[x][j - 1];
            int h = -1;
            for (int k = 1; k < j; ++k) {
                const double c = cost(l, k) + cost(r, j - k);
                if (c < d) {
                    d = c;
                    h = k;
                }
            }
            D_[x][j] = d;
            how_[x][j] = h;
        }
    }
    // the binary subtrees (or leaves) that cover slot s with at most j slots
    void cover(const Slot& s, int j, std::vector<Slot>& out) const {
        if (s.ref < 0) {
            out.push_back(s);
            return;
        }
        while (j > 1 && how_[s.ref][j] == -1) --j;
        if (j == 1 || how_[s.ref][j] == 0) {
            out.push_back(s);
            return;
        }
        const int k = how_[s.ref][j];
        cover(slot(s.ref, 0), k, out);
        cover(slot(s.ref, 1), j - k, out);
    }
    // 4-wide node for binary node x, at most `budget` pushes on any path
    // from it down (need_[x] <= budget holds on entry)
    int32_t build(int32_t x, int budget, int pushed) {
        const Slot l = slot(x, 0), r = slot(x, 1);
        std::vector<Slot> c, trial;
        double best = INFINITY;
        for (int total = 2; total <= 4; ++total) {
            for (int k = 1; k < total; ++k) {
                trial.clear();
                cover(l, k, trial);
                cover(r, total - k, trial);
                const int left = budget - ((int)trial.size() - 1);
                bool fits = true;
                for (const Slot& t : trial) fits = fits && need(t) <= left;
                const double cst = cost(l, k) + cost(r, total - k);
                if (fits && cst < best) {
                    best = cst;
                    c = trial;
                }
            }
        }
        if (c.empty()) c = {l, r};   // unreachable: two children always fit
        const int32_t idx = (int32_t)b_->wide4.size();
        b_->wide4.push_back(Wide4{});
        const int pushes = (int)c.size() - 1;
        int32_t refs[4];
        for (int i = 0; i < (int)c.size(); ++i) {
            if (c[i].ref >= 0) {
                refs[i] = build(c[i].ref, budget - pushes, pushed + pushes);
            } else {
                refs[i] = c[i].ref;
                max_push_ = std::max(max_push_, pushed + pushes);
            }
        }
        Wide4& nd = b_->wide4[idx];
        for (int i = 0; i < 4; ++i) {
            if (i < (int)c.size()) {
                for (int k = 0; k < 3; ++k) {
                    nd.lo[k][i] = c[i].lo[k];
                    nd.hi[k][i] = c[i].hi[k];
                }
                nd.child[i] = refs[i];
            } else {
                for (int k = 0; k < 3; ++k) {
                    nd.lo[k][i] = INFINITY;
                    nd.hi[k][i] = -INFINITY;
                }
                nd.child[i] = kEmptyChild;
            }
        }
        return idx;
    }
};
// Expected traversal cost of a 4-wide tree in the units of OptimalCollapser:
// every node is entered with probability (its box area / the root's), costing
// one node step; every leaf, likewise, costs kTriCost per triangle.
double sah_cost4(const std::vector<Wide4>& nodes) {
    auto area = [](const float* lo, const float* hi) {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = std::max(0.0, (double)hi[k] - (double)lo[k]);
        return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
    };
    const Wide4& r = nodes[0];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < 4; ++i) {
        if (r.child[i] == kEmptyChild) continue;
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], r.lo[k][i]);
            hi[k] = std::max(hi[k], r.hi[k][i]);
        }
    }
    // area ratios are scale-free: only a root of zero area needs a stand-in
    const double root_area = area(lo, hi);
    const double root = root_area > 0.0 ? root_area : 1.0;
    double c = OptimalCollapser::kNodeCost;
    for (const Wide4& n : nodes) {
        for (int i = 0; i < 4; ++i) {
            if (n.child[i] == kEmptyChild) continue;
            const float sl[3] = {n.lo[0][i], n.lo[1][i], n.lo[2][i]};
            const float sh[3] = {n.hi[0][i], n.hi[1][i], n.hi[2][i]};
            const double p = area(sl, sh) / root;
            c += n.child[i] >= 0 ? p * OptimalCollapser::kNodeCost
                                 : p * OptimalCollapser::kTriCost * (((~n.child[i]) & 7) + 1);
        }
    }
    return c;
}

// ---- the device encoding of the 4-wide nodes --------------------------------
double half_value(uint16_t h) {   // non-negative finite halves only
    const int e = (h >> 10) & 31, m = h & 1023;
    return e == 0 ? std::ldexp((double)m, -24) : std::ldexp((double)(1024 + m), e - 25);
}

// The half nearest to v (0 <= v <= 65504), then stepped to the largest half
// <= v (up = false) or the smallest half >= v (up = true).  Bit patterns of
// non-negative halves increase with their values.
uint16_t half_bound(double v, bool up) {
    uint16_t h;
    if (v < 6.103515625e-05) {
        h = (uint16_t)std::llround(v * 16777216.0);   // subnormal step 2^-24
    } else {
        int ex;
        const double fr = std::frexp(v, &ex);           // v = fr 2^ex, fr in [0.5, 1)
        long m = std::llround((fr * 2.0 - 1.0) * 1024.0);
        int E = ex - 1 + 15;
        if (m == 1024) {
            m = 0;
            ++E;
        }
        h = (uint16_t)((E << 10) | m);
    }
    if (up) {
        while (half_value(h) < v) ++h;
    } else {
        while (h > 0 && half_value(h) > v) --h;
    }
    return h;
}

// signed directed rounding: largest half <= v (up = false) or smallest >= v
uint16_t half_bound_signed(double v, bool up) {
    if (v >= 0.0) return half_bound(v, up);
    return (uint16_t)(0x8000u | half_bound(-v, !up));
}

// Per axis, the origin is the low bound of the thinnest used child, whose
// bounds then encode almost exactly (flat walls stay thin).
double node_origin(const Wide4& w, int k) {
    double org = 0.0, thin = INFINITY;
    for (int i = 0; i < 4; ++i) {
        if (w.child[i] == kEmptyChild) continue;
        const double t = (double)w.hi[k][i] - (double)w.lo[k][i];
        if (t < thin) {
            thin = t;
            org = w.lo[k][i];
        }
    }
    return org;
}

// The scene-wide exponent E of the half-precision offsets: every offset
// from a node origin, in units of 2^E, stays within the half range (2^15 <
// 65504).  A half carries 11 significant bits wherever it is normal, so one
// exponent for the whole tree loses nothing against one per node; offsets
// below 2^(E-14) fall into the subnormal range and are still rounded
// outward.  E is kept large enough that the scaled origins are normal
// single-precision numbers.
int box_exponent(const std::vector<Wide4>& nodes) {
    double span = 0.0, mag = 0.0;
    for (const Wide4& w : nodes)
        for (int k = 0; k < 3; ++k) {
            const double org = node_origin(w, k);
            for (int i = 0; i < 4; ++i) {
                if (w.child[i] == kEmptyChild) continue;
                span = std::max(span, std::max(org - (double)w.lo[k][i], (double)w.hi[k][i] - org));
                mag = std::max(mag, std::fabs(org));
            }
        }
    int e = span > 0.0 ? (int)std::ceil(std::log2(span)) - 15 : -30;
    if (mag > 0.0) e = std::max(e, (int)std::ceil(std::log2(mag)) - 120);
    return std::min(std::max(e, -120), 100);
}

Bvh4Node encode4(const Wide4& w, int e) {
    Bvh4Node n;
    std::memset(&n, 0, sizeof(n));
    for (int k = 0; k < 3; ++k) {
        // the stored origin, in units of 2^e (exact: a power-of-two scaling
        // of a normal number); offsets are taken from it as stored
        n.org[k] = (float)std::ldexp(node_origin(w, k), -e);
        const double org = (double)n.org[k];
        for (int i = 0; i < 4; ++i) {
            if (w.child[i] == kEmptyChild) {
                n.q[k][i] = 0x7C00;       // +inf
                n.q[k][4 + i] = 0xFC00;   // -inf
                continue;
            }
            n.q[k][i] = half_bound_signed(std::ldexp((double)w.lo[k][i], -e) - org, false);
            n.q[k][4 + i] = half_bound_signed(std::ldexp((double)w.hi[k][i], -e) - org, true);
        }
    }
    for (int i = 0; i < 4; ++i) n.child[i] = node4_ref(w.child[i]);
    return n;
}

}  // namespace

int build_bvh(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
              HostBvh* out) {
    if (n_tris < 1 || n_tris >= (int64_t(1) << 28))
        return fail(FIPT_EINVAL, "n_tris must be in [1, 2^28), got %lld", (long long)n_tris);
    for (int64_t i = 0; i < 3 * n_tris; ++i)
        if (tris[i] < 0 || tris[i] >= n_verts)
            return fail(FIPT_EINVAL, "triangle %lld references vertex %d outside [0, %lld)",
                        (long long)(i / 3), tris[i], (long long)n_verts);
    for (int64_t i = 0; i < 3 * n_verts; ++i)
        if (!std::isfinite(verts[i]))
            return fail(FIPT_EINVAL, "vertex %lld has a non-finite coordinate", (long long)(i / 3));
    Builder bld(verts, tris, n_tris, out);
    bld.run();
    if (out->max_depth > kMaxInnerDepth)
        return fail(FIPT_EINVAL, "BVH depth %d exceeds the traversal stack", out->max_depth);
    // two collapses under the stack budget; keep the one of lower expected
    // cost (the surface-area-guided one wins unless the binary tree is so
    // deep that the budget forces narrow nodes near the root)
    OptimalCollapser opt(out);
    opt.run();
    std::vector<Wide4> guided;
    guided.swap(out->wide4);
    const int guided_push = out->max_push4;
    Collapser greedy(out);
    greedy.run();
    if (sah_cost4(guided) < sah_cost4(out->wide4)) {
        out->wide4.swap(guided);
        out->max_push4 = guided_push;
    }
    out->box_exp = box_exponent(out->wide4);
    out->nodes4.resize(out->wide4.size());
    for (size_t i = 0; i < out->wide4.size(); ++i)
        out->nodes4[i] = encode4(out->wide4[i], out->box_exp);
    if (out->max_push4 > kStackSize)
        return fail(FIPT_EINVAL, "4-wide BVH needs %d stack entries", out->max_push4);
    // the traversal addresses nodes by non-negative 32-bit byte offsets
    if ((int64_t)out->nodes4.size() > kMaxNodes4)
        return fail(FIPT_EINVAL, "4-wide BVH has %zu nodes (at most %lld)", out->nodes4.size(),
                    (long long)kMaxNodes4);
    return FIPT_OK;
}

}  // namespace fipt

namespace {

// Walk the 4-wide node `idx`: every used slot's single-precision box
// encloses the boxes of the child node (up to the widening margin) or the
// vertices of the leaf's triangles, its decoded device box (origin plus
// half-precision offsets) encloses the single-precision one, unused slots
// encode an inverted box; count triangle occurrences and the stack pushes
// on each path.
int validate4(const fipt::HostBvh& b, const float* verts, const int32_t* tris, int32_t idx,
              int pushed, std::vector<int>& seen, int* max_push) {
    using namespace fipt;
    if (idx < 0 || idx >= (int32_t)b.nodes4.size() || b.nodes4.size() != b.wide4.size())
        return fail(FIPT_EINVAL, "4-wide child index %d out of range", idx);
    const Wide4& nd = b.wide4[idx];
    const Bvh4Node& en = b.nodes4[idx];
    int used = 0;
    for (int i = 0; i < 4; ++i) {
        if (en.child[i] != node4_ref(nd.child[i]))
            return fail(FIPT_EINVAL, "4-wide node %d: child mismatch", idx);
        if (nd.child[i] != kEmptyChild) {
            ++used;
            continue;
        }
        // the traversal relies on unused slots holding an inverted box
        for (int k = 0; k < 3; ++k)
            if (en.q[k][i] != 0x7C00 || en.q[k][4 + i] != 0xFC00)
                return fail(FIPT_EINVAL, "4-wide node %d: unused slot %d has a box", idx, i);
    }
    if (used < 1) return fail(FIPT_EINVAL, "4-wide node %d has no children", idx);
    const int here = pushed + used - 1;
    for (int i = 0; i < 4; ++i) {
        const int32_t c = nd.child[i];
        if (c == kEmptyChild) continue;
        const float lo[3] = {nd.lo[0][i], nd.lo[1][i], nd.lo[2][i]};
        const float hi[3] = {nd.hi[0][i], nd.hi[1][i], nd.hi[2][i]};
        for (int k = 0; k < 3; ++k) {
            auto sv = [](uint16_t h) { return (h & 0x8000u) ? -half_value(h & 0x7FFFu) : half_value(h); };
            const double dlo = std::ldexp((double)en.org[k] + sv(en.q[k][i]), b.box_exp);
            const double dhi = std::ldexp((double)en.org[k] + sv(en.q[k][4 + i]), b.box_exp);
            if (!(dlo <= (double)lo[k] && dhi >= (double)hi[k]))
                return fail(FIPT_EINVAL, "4-wide node %d: encoded slot %d does not enclose its box", idx, i);
        }
        if (c >= 0) {
            const Wide4& ch = b.wide4[c];
            for (int j = 0; j < 4; ++j) {
                if (ch.child[j] == kEmptyChild) continue;
                for (int k = 0; k < 3; ++k) {
                    const float tol = 4.0f * 9.5367431640625e-07f *
                                          std::max(std::fabs(lo[k]), std::fabs(hi[k])) + 1.17549435e-38f;
                    if (ch.lo[k][j] < lo[k] - tol || ch.hi[k][j] > hi[k] + tol)
                        return fail(FIPT_EINVAL, "4-wide node %d leaves its parent box", c);
                }
            }
            int rc = validate4(b, verts, tris, c, here, seen, max_push);
            if (rc) return rc;
        } else {
            const int32_t lr = ~c;
            const int64_t first = lr >> 3;
            const int cnt = (lr & 7) + 1;
            if (first + cnt > (int64_t)b.tris.size()) return fail(FIPT_EINVAL, "leaf range out of bounds");
            for (int t = 0; t < cnt; ++t) {
                const int32_t f = b.order[first + t];
                ++seen[f];
                for (int v = 0; v < 3; ++v) {
                    const float* p = verts + 3 * (int64_t)tris[3 * (int64_t)f + v];
                    for (int k = 0; k < 3; ++k)
                        if (p[k] < lo[k] || p[k] > hi[k])
                            return fail(FIPT_EINVAL, "triangle %d pokes out of its 4-wide leaf box", f);
                }
            }
            *max_push = std::max(*max_push, here);
        }
    }
    return FIPT_OK;
}

// Walk the subtree of `ref`: count triangle occurrences, check that the
// box recorded for `ref` in its parent encloses all of its triangles, and
// track the deepest internal node.
int validate_subtree(const fipt::HostBvh& b, const float* verts, const int32_t* tris,
                     int32_t ref, const float lo[3], const float hi[3], int depth,
                     std::vector<int>& seen, int* max_depth) {
    using namespace fipt;
    if (ref >= 0) {
        if (ref >= (int32_t)b.nodes.size()) return fail(FIPT_EINVAL, "child index %d out of range", ref);
        if (depth > kMaxInnerDepth) return fail(FIPT_EINVAL, "internal node at depth %d", depth);
        *max_depth = std::max(*max_depth, depth);
        const BvhNode& nd = b.nodes[ref];
        const float l0[3] = {nd.c0lx, nd.c0ly, nd.c0lz}, h0[3] = {nd.c0hx, nd.c0hy, nd.c0hz};
        const float l1[3] = {nd.c1lx, nd.c1ly, nd.c1lz}, h1[3] = {nd.c1hx, nd.c1hy, nd.c1hz};
        for (int k = 0; k < 3; ++k)
            if (l0[k] < lo[k] || h0[k] > hi[k] || l1[k] < lo[k] || h1[k] > hi[k]) {
                // children are widened independently of the parent; allow
                // their few-ulp margin
                const float tol = 4.0f * 9.5367431640625e-07f * std::max(std::fabs(lo[k]), std::fabs(hi[k])) + 1.17549435e-38f;
                if (l0[k] < lo[k] - tol || h0[k] > hi[k] + tol || l1[k] < lo[k] - tol || h1[k] > hi[k] + tol)
                    return fail(FIPT_EINVAL, "child box of node %d leaves its parent box", ref);
            }
        int rc = validate_subtree(b, verts, tris, nd.child0, l0, h0, depth + 1, seen, max_depth);
        if (rc) return rc;
        // a one-triangle scene references the same leaf twice
        if (nd.child1 == nd.child0 && ref == 0 && b.tris.size() == 1) return FIPT_OK;
        return validate_subtree(b, verts, tris, nd.child1, l1, h1, depth + 1, seen, max_depth);
    }
    const int32_t lr = ~ref;
    const int64_t first = lr >> 3;
    const int cnt = (lr & 7) + 1;
    if (first + cnt > (int64_t)b.tris.size()) return fail(FIPT_EINVAL, "leaf range out of bounds");
    for (int i = 0; i < cnt; ++i) {
        const int32_t f = b.order[first + i];
        if (b.tris[first + i].orig != f) return fail(FIPT_EINVAL, "leaf triangle id mismatch");
        ++seen[f];
        for (int v = 0; v < 3; ++v) {
            const float* p = verts + 3 * (int64_t)tris[3 * (int64_t)f + v];
            for (int k = 0; k < 3; ++k)
                if (p[k] < lo[k] || p[k] > hi[k])
                    return fail(FIPT_EINVAL, "triangle %d pokes out of its leaf box", f);
        }
    }
    return FIPT_OK;
}

}  // namespace

extern "C" int fipt_bvh_validate(const float* verts, int64_t n_verts, const int32_t* tris,
                                 int64_t n_tris, int64_t* n_nodes, int32_t* max_depth) {
    using namespace fipt;
    clear_error();
    if (!verts || !tris || !n_nodes || !max_depth) return fail(FIPT_EINVAL, "NULL argument");
    if (n_verts < 3) return fail(FIPT_EINVAL, "n_verts must be >= 3");
    HostBvh b;
    int rc = build_bvh(verts, n_verts, tris, n_tris, &b);
    if (rc) return rc;
    std::vector<int> seen(n_tris, 0);
    int depth = 0;
    const float lo[3] = {-INFINITY, -INFINITY, -INFINITY}, hi[3] = {INFINITY, INFINITY, INFINITY};
    rc = validate_subtree(b, verts, tris, 0, lo, hi, 0, seen, &depth);
    if (rc) return rc;
    for (int64_t f = 0; f < n_tris; ++f)
        if (seen[f] != 1) return fail(FIPT_EINVAL, "triangle %lld appears %d times", (long long)f, seen[f]);
    if ((int64_t)b.tris.size() != n_tris) return fail(FIPT_EINVAL, "leaf order has %zu triangles", b.tris.size());
    // the 4-wide tree the GPU traverses
    std::vector<int> seen4(n_tris, 0);
    int pushes = 0;
    rc = validate4(b, verts, tris, 0, 0, seen4, &pushes);
    if (rc) return rc;
    for (int64_t f = 0; f < n_tris; ++f)
        if (seen4[f] != (n_tris == 1 ? 2 : 1))
            return fail(FIPT_EINVAL, "4-wide tree: triangle %lld appears %d times", (long long)f, seen4[f]);
    if (pushes > kStackSize || pushes != b.max_push4)
        return fail(FIPT_EINVAL, "4-wide tree needs %d stack entries (builder said %d)", pushes, b.max_push4);
    *n_nodes = (int64_t)b.nodes4.size();
    *max_depth = depth;
    return FIPT_OK;
}
