// Host-side builder of the 4-wide bounding-volume hierarchy.
//
// Binned surface-area-heuristic splits (32 bins on the widest centroid axis)
// build a binary tree, subtrees above 64k triangles in parallel; the binary
// tree is then collapsed into 4-wide nodes by repeatedly opening the child
// with the largest surface area, and linearised depth-first.  If the 4-wide
// tree would be too deep for the traversal stack, the build is redone with
// object-median splits, which bounds the depth by log2 of the triangle count.
#include "bvh_build.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <future>
#include <memory>
#include <thread>
#include <vector>

namespace ocr {
namespace {

struct Box {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const Box &b) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], b.lo[a]);
            hi[a] = std::max(hi[a], b.hi[a]);
        }
    }
    void grow(const float *p) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p[a]);
            hi[a] = std::max(hi[a], p[a]);
        }
    }
    float area() const {
        float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        if (!(dx >= 0.f) || !(dy >= 0.f) || !(dz >= 0.f)) return 0.f;
        return 2.f * (dx * dy + dy * dz + dz * dx);
    }
};

struct Prim {
    Box box;
    float c[3];
};

struct BNode {  // binary node
    Box box;
    int32_t left = -1, right = -1;  // children (indices into the task's node vector)
    int32_t first = 0, count = 0;   // leaf range into the permutation
};

struct Tree {
    std::vector<BNode> nodes;
};

constexpr int kBins = 32;
constexpr float kTrav = 1.0f, kIsect = 1.0f;

class Builder {
   public:
    Builder(const std::vector<Prim> &prims, bool median) : prims_(prims), median_(median) {
        perm_.resize(prims.size());
        for (size_t i = 0; i < perm_.size(); ++i) perm_[i] = (uint32_t)i;
    }

    // Returns root index in tree_.
    int32_t build() {
        tree_.nodes.reserve(prims_.size() / 2 + 16);
        return build_rec(tree_, 0, (int32_t)prims_.size(), 0);
    }

    const std::vector<uint32_t> &perm() const { return perm_; }
    Tree &tree() { return tree_; }

   private:
    int32_t build_rec(Tree &t, int32_t first, int32_t count, int depth) {
        Box box, cbox;
        for (int32_t i = first; i < first + count; ++i) {
            const Prim &p = prims_[perm_[i]];
            box.grow(p.box);
            cbox.grow(p.c);
        }
        int32_t id = (int32_t)t.nodes.size();
        t.nodes.emplace_back();
        t.nodes[id].box = box;
        if (count <= 2) {
            t.nodes[id].first = first;
            t.nodes[id].count = count;
            return id;
        }
        int axis = 0;
        float ext[3];
        for (int a = 0; a < 3; ++a) ext[a] = cbox.hi[a] - cbox.lo[a];
        if (ext[1] > ext[axis]) axis = 1;
        if (ext[2] > ext[axis]) axis = 2;
        int32_t mid = -1;
        if (!(ext[axis] > 0.f)) {
            if (count <= kMaxLeaf) {
                t.nodes[id].first = first;
                t.nodes[id].count = count;
                return id;
            }
            mid = first + count / 2;
        } else if (median_) {
            mid = first + count / 2;
            std::nth_element(perm_.begin() + first, perm_.begin() + mid, perm_.begin() + first + count,
                             [&](uint32_t a, uint32_t b) { return prims_[a].c[axis] < prims_[b].c[axis]; });
            if (count <= 4) {
                t.nodes[id].first = first;
                t.nodes[id].count = count;
                return id;
            }
        } else {
            Box bb[kBins];
            int32_t bn[kBins] = {0};
            float scale = kBins / ext[axis];
            auto bin_of = [&](const Prim &p) {
                int b = (int)((p.c[axis] - cbox.lo[axis]) * scale);
                return std::min(std::max(b, 0), kBins - 1);
            };
            for (int32_t i = first; i < first + count; ++i) {
                const Prim &p = prims_[perm_[i]];
                int b = bin_of(p);
                bb[b].grow(p.box);
                bn[b]++;
            }
            float rarea[kBins];
            int32_t rcount[kBins];
            Box acc;
            int32_t n = 0;
            for (int b = kBins - 1; b > 0; --b) {
                acc.grow(bb[b]);
                n += bn[b];
                rarea[b] = acc.area();
                rcount[b] = n;
            }
            Box lacc;
            int32_t ln = 0;
            float best = INFINITY;
            int best_b = -1;
            float parea = box.area();
            for (int b = 1; b < kBins; ++b) {
                lacc.grow(bb[b - 1]);
                ln += bn[b - 1];
                if (ln == 0 || rcount[b] == 0) continue;
                float cost = kTrav + kIsect * (lacc.area() * ln + rarea[b] * rcount[b]) / std::max(parea, 1e-30f);
                if (cost < best) {
                    best = cost;
                    best_b = b;
                }
            }
            float leaf_cost = kIsect * count;
            if (count <= kMaxLeaf && (best_b < 0 || leaf_cost <= best)) {
                t.nodes[id].first = first;
                t.nodes[id].count = count;
                return id;
            }
            if (best_b < 0) {
                mid = first + count / 2;
            } else {
                auto it = std::partition(perm_.begin() + first, perm_.begin() + first + count,
                                         [&](uint32_t a) { return bin_of(prims_[a]) < best_b; });
                mid = (int32_t)(it - perm_.begin());
                if (mid == first || mid == first + count) mid = first + count / 2;
            }
        }
        int32_t lc = mid - first, rc = count - lc;
        int32_t l, r;
        if (count > 65536 && depth < 12) {
            // Build the right subtree on another thread into its own tree,
            // then splice it in.
            Tree sub;
            sub.nodes.reserve(rc / 2 + 16);
            auto fut = std::async(std::launch::async, [&] { return build_rec(sub, mid, rc, depth + 1); });
            l = build_rec(t, first, lc, depth + 1);
            int32_t sroot = fut.get();
            int32_t base = (int32_t)t.nodes.size();
            for (BNode nd : sub.nodes) {
                if (nd.left >= 0) {
                    nd.left += base;
                    nd.right += base;
                }
                t.nodes.push_back(nd);
            }
            r = base + sroot;
        } else {
            l = build_rec(t, first, lc, depth + 1);
            r = build_rec(t, mid, rc, depth + 1);
        }
        t.nodes[id].left = l;
        t.nodes[id].right = r;
        return id;
    }

    const std::vector<Prim> &prims_;
    bool median_;
    std::vector<uint32_t> perm_;
    Tree tree_;
};

struct Flattener {
    const std::vector<BNode> &bn;
    const std::vector<uint32_t> &perm;
    const float *V;
    const uint32_t *F;
    std::vector<Node4> nodes;
    std::vector<float4> tris;
    int max_depth = 0;
    int max_leaf = 0;

    uint32_t leaf_link(const BNode &n) {
        uint32_t first = (uint32_t)(tris.size() / 3);
        for (int32_t i = 0; i < n.count; ++i) {
            uint32_t t = perm[n.first + i];
            for (int k = 0; k < 3; ++k) {
                const float *p = V + 3 * (size_t)F[3 * (size_t)t + k];
                float4 v;
                v.x = p[0];
                v.y = p[1];
                v.z = p[2];
                uint32_t idw = k == 0 ? t : 0u;
                std::memcpy(&v.w, &idw, 4);
                tris.push_back(v);
            }
        }
        max_leaf = std::max(max_leaf, (int)n.count);
        return kLeafBit | ((uint32_t)(n.count - 1) << 27) | first;
    }

    // Emit the 4-wide node for binary node b; returns its index.
    uint32_t emit(int32_t b, int depth) {
        max_depth = std::max(max_depth, depth);
        int32_t kids[4];
        int nk = 0;
        const BNode &root = bn[b];
        kids[nk++] = root.left;
        kids[nk++] = root.right;
        while (nk < 4) {
            int best = -1;
            float ba = -1.f;
            for (int i = 0; i < nk; ++i) {
                const BNode &c = bn[kids[i]];
                if (c.count == 0 && c.left >= 0 && c.box.area() > ba) {
                    ba = c.box.area();
                    best = i;
                }
            }
            if (best < 0) break;
            int32_t open = kids[best];
            kids[best] = bn[open].left;
            kids[nk++] = bn[open].right;
        }
        uint32_t me = (uint32_t)nodes.size();
        nodes.emplace_back();
        Node4 nd;
        for (int i = 0; i < 4; ++i) {
            nd.lox[i] = nd.loy[i] = nd.loz[i] = INFINITY;
            nd.hix[i] = nd.hiy[i] = nd.hiz[i] = -INFINITY;
            nd.child[i] = kEmpty;
            nd.pad[i] = 0;
        }
        for (int i = 0; i < nk; ++i) {
            const BNode &c = bn[kids[i]];
            nd.lox[i] = c.box.lo[0];
            nd.loy[i] = c.box.lo[1];
            nd.loz[i] = c.box.lo[2];
            nd.hix[i] = c.box.hi[0];
            nd.hiy[i] = c.box.hi[1];
            nd.hiz[i] = c.box.hi[2];
            if (c.left < 0) nd.child[i] = leaf_link(c);
            else nd.child[i] = emit(kids[i], depth + 1);
        }
        nodes[me] = nd;
        return me;
    }
};

}  // namespace

int build_bvh_host(const float *V, int64_t nv, const uint32_t *F, int64_t nt, HostBVH &out) {
    (void)nv;
    auto t0 = std::chrono::steady_clock::now();
    std::vector<Prim> prims((size_t)nt);
    for (int64_t t = 0; t < nt; ++t) {
        Prim &p = prims[(size_t)t];
        for (int k = 0; k < 3; ++k) p.box.grow(V + 3 * (size_t)F[3 * t + k]);
        for (int a = 0; a < 3; ++a) p.c[a] = 0.5f * (p.box.lo[a] + p.box.hi[a]);
    }
    for (int attempt = 0; attempt < 2; ++attempt) {
        Builder b(prims, attempt == 1);
        int32_t root = b.build();
        const std::vector<BNode> &bn = b.tree().nodes;
        Flattener fl{bn, b.perm(), V, F, {}, {}, 0, 0};
        fl.nodes.reserve(bn.size() / 3 + 4);
        fl.tris.reserve((size_t)nt * 3);
        if (bn[root].left < 0) {
            // single leaf: wrap it in one node
            Node4 nd;
            for (int i = 0; i < 4; ++i) {
                nd.lox[i] = nd.loy[i] = nd.loz[i] = INFINITY;
                nd.hix[i] = nd.hiy[i] = nd.hiz[i] = -INFINITY;
                nd.child[i] = kEmpty;
                nd.pad[i] = 0;
            }
            const BNode &c = bn[root];
            nd.lox[0] = c.box.lo[0];
            nd.loy[0] = c.box.lo[1];
            nd.loz[0] = c.box.lo[2];
            nd.hix[0] = c.box.hi[0];
            nd.hiy[0] = c.box.hi[1];
            nd.hiz[0] = c.box.hi[2];
            fl.nodes.push_back(nd);
            fl.nodes[0].child[0] = fl.leaf_link(c);
            fl.max_depth = 1;
        } else {
            fl.emit(root, 1);
        }
        if (fl.max_depth <= kMaxDepth || attempt == 1) {
            out.nodes = std::move(fl.nodes);
            out.tris = std::move(fl.tris);
            out.depth = fl.max_depth;
            out.max_leaf = fl.max_leaf;
            out.median_fallback = attempt == 1;
            break;
        }
    }
    auto t1 = std::chrono::steady_clock::now();
    out.build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return out.depth <= kMaxDepth ? 0 : -1;
}

}  // namespace ocr
