// Host-side BVH builder interface.
#pragma once

#include <vector>

#include "ocr_common.hpp"

namespace ocr {

struct HostBVH {
    std::vector<Node4> nodes;
    std::vector<float4> tris;  // 3 per triangle, leaf order
    int depth = 0;
    int max_leaf = 0;
    bool median_fallback = false;
    double build_ms = 0.0;
};

// Returns 0 on success, -1 if the tree is deeper than the traversal stack
// allows even after the object-median fallback.
int build_bvh_host(const float *V, int64_t nv, const uint32_t *F, int64_t nt, HostBVH &out);

}  // namespace ocr
