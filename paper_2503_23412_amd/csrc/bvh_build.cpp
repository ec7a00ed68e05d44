// Host-side BVH construction: binned SAH binary tree (16 bins, three axes), collapsed into
// 4-wide nodes of one 128-byte line each and, on request, into 8-wide nodes with quantised child
// boxes, also one line each (the child with the largest surface area is opened until the width
// is reached). Triangles are reordered so that every leaf is one contiguous range of at most 4
// triangles; both trees share the leaves, hence the triangle order.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "pt_layout.h"

namespace ptbvh {

struct Box {
    float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    void grow(const Box &b)
    {
        for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], b.lo[k]); hi[k] = std::max(hi[k], b.hi[k]); }
    }
    void grow(const float *p)
    {
        for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], p[k]); hi[k] = std::max(hi[k], p[k]); }
    }
    float area() const
    {
        if (lo[0] > hi[0]) return 0.0f;
        const float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        return 2.0f * (dx * dy + dy * dz + dz * dx);
    }
};

struct BinNode {
    Box box;
    int left = -1, right = -1;   // children (binary), -1 for a leaf
    int first = 0, count = 0;    // leaf range in the reordered reference array
};

struct Builder {
    std::vector<Box> tbox;
    std::vector<float> cent;     // 3 per triangle
    std::vector<int> ref;
    std::vector<BinNode> nodes;

    int build(int first, int count)
    {
        const int id = (int)nodes.size();
        nodes.emplace_back();
        Box b, cb;
        for (int i = first; i < first + count; ++i) { b.grow(tbox[ref[i]]); cb.grow(&cent[3 * ref[i]]); }
        nodes[id].box = b;
        if (count <= 4) { nodes[id].first = first; nodes[id].count = count; return id; }
        // binned SAH
        const int NB = 16;
        float best = FLT_MAX;
        int best_axis = -1, best_split = -1;
        for (int ax = 0; ax < 3; ++ax) {
            const float lo = cb.lo[ax], ext = cb.hi[ax] - cb.lo[ax];
            if (!(ext > 0.0f)) continue;
            Box bb[NB];
            int bc[NB] = {0};
            for (int i = first; i < first + count; ++i) {
                int k = (int)((cent[3 * ref[i] + ax] - lo) / ext * NB);
                k = std::min(std::max(k, 0), NB - 1);
                bb[k].grow(tbox[ref[i]]);
                bc[k]++;
            }
            Box la[NB];
            int lc[NB];
            Box acc;
            int n = 0;
            for (int k = 0; k < NB; ++k) { acc.grow(bb[k]); n += bc[k]; la[k] = acc; lc[k] = n; }
            Box racc;
            int rn = 0;
            for (int k = NB - 1; k > 0; --k) {
                racc.grow(bb[k]); rn += bc[k];
                const int ln = lc[k - 1];
                if (ln == 0 || rn == 0) continue;
                const float c = la[k - 1].area() * ln + racc.area() * rn;
                if (c < best) { best = c; best_axis = ax; best_split = k; }
            }
        }
        int mid;
        if (best_axis < 0) {
            mid = first + count / 2;   // all centroids coincide: split the range in halves
        } else {
            const float lo = cb.lo[best_axis], ext = cb.hi[best_axis] - cb.lo[best_axis];
            auto it = std::partition(ref.begin() + first, ref.begin() + first + count, [&](int t) {
                int k = (int)((cent[3 * t + best_axis] - lo) / ext * NB);
                k = std::min(std::max(k, 0), NB - 1);
                return k < best_split;
            });
            mid = (int)(it - ref.begin());
            if (mid == first || mid == first + count) mid = first + count / 2;
        }
        const int l = build(first, mid - first);
        const int r = build(mid, first + count - mid);
        nodes[id].left = l;
        nodes[id].right = r;
        return id;
    }
};

static void set_child(BNode &n, int k, const Box &b, int child, int count)
{
    n.lo_x[k] = b.lo[0]; n.hi_x[k] = b.hi[0];
    n.lo_y[k] = b.lo[1]; n.hi_y[k] = b.hi[1];
    n.lo_z[k] = b.lo[2]; n.hi_z[k] = b.hi[2];
    n.child[k] = child; n.count[k] = count;
}

// collapse binary node `bn` into wide node index `wi` of `out`
static std::vector<int> open_children(const Builder &B, int bn, int w);
static void collapse(const Builder &B, int bn, std::vector<BNode> &out, int wi)
{
    const std::vector<int> kids = open_children(B, bn, 4);
    BNode n;
    std::memset(&n, 0, sizeof(n));
    for (int k = 0; k < 4; ++k) {
        n.lo_x[k] = n.lo_y[k] = n.lo_z[k] = FLT_MAX;
        n.hi_x[k] = n.hi_y[k] = n.hi_z[k] = -FLT_MAX;
        n.child[k] = -1; n.count[k] = -1;
    }
    std::vector<std::pair<int, int>> inner;   // (slot, binary node)
    for (int k = 0; k < (int)kids.size(); ++k) {
        const BinNode &c = B.nodes[kids[k]];
        if (c.left < 0) set_child(n, k, c.box, c.first, c.count);
        else inner.push_back({k, kids[k]});
    }
    for (auto &pr : inner) {
        const int idx = (int)out.size();
        out.emplace_back();
        set_child(n, pr.first, B.nodes[pr.second].box, idx, 0);
    }
    out[wi] = n;
    for (auto &pr : inner) collapse(B, pr.second, out, out[wi].child[pr.first]);
}

// the children of binary node `bn` in a node of width w: open the child of largest area until w
static std::vector<int> open_children(const Builder &B, int bn, int w)
{
    std::vector<int> kids;
    const BinNode &root = B.nodes[bn];
    if (root.left < 0) kids.push_back(bn);
    else { kids.push_back(root.left); kids.push_back(root.right); }
    while ((int)kids.size() < w) {
        int pick = -1;
        float pa = -1.0f;
        for (int i = 0; i < (int)kids.size(); ++i) {
            const BinNode &c = B.nodes[kids[i]];
            if (c.left >= 0 && c.box.area() > pa) { pa = c.box.area(); pick = i; }
        }
        if (pick < 0) break;
        const int c = kids[pick];
        kids.erase(kids.begin() + pick);
        kids.push_back(B.nodes[c].left);
        kids.push_back(B.nodes[c].right);
    }
    return kids;
}

// quantisation of one axis of an 8-wide node: the scale 2^k is the smallest power of two with
// (hi - lo) / 2^k <= 255, the grid starts at lo; planes round outwards (checked in float, the
// precision the traversal decodes them in, and stepped one more cell out when rounding there
// would cut into the box)
static void quant_axis(float lo, float hi, float &org, uint8_t &ebits, float &scale)
{
    org = lo;
    const double ext = std::max((double)hi - (double)lo, 0.0);
    int k = -126;
    if (ext > 0.0) k = std::max(-126, (int)std::ceil(std::log2(ext / 255.0)));
    while (std::ldexp(255.0, k) < ext) ++k;
    scale = std::ldexp(1.0f, k);
    ebits = (uint8_t)(k + 127);
}
static uint8_t q_lo(float v, float org, float scale)
{
    int q = (int)std::floor(((double)v - (double)org) / (double)scale);
    q = std::min(std::max(q, 0), 255);
    while (q > 0 && org + (float)q * scale > v) --q;
    return (uint8_t)q;
}
static uint8_t q_hi(float v, float org, float scale)
{
    int q = (int)std::ceil(((double)v - (double)org) / (double)scale);
    q = std::min(std::max(q, 0), 255);
    while (q < 255 && org + (float)q * scale < v) ++q;
    return (uint8_t)q;
}

// collapse binary node `bn` into 8-wide node index `wi` of `out`
static void collapse8(const Builder &B, int bn, std::vector<BNode8> &out, int wi)
{
    const std::vector<int> kids = open_children(B, bn, 8);
    BNode8 n;
    std::memset(&n, 0, sizeof(n));
    Box nb;
    for (int c : kids) nb.grow(B.nodes[c].box);
    float org[3], sc[3];
    for (int a = 0; a < 3; ++a) quant_axis(nb.lo[a], nb.hi[a], org[a], n.e[a], sc[a]);
    for (int a = 0; a < 3; ++a) n.org[a] = org[a];
    for (int k = 0; k < 8; ++k) { n.child[k] = -1; n.count[k] = PT_CHILD_EMPTY; }
    std::vector<std::pair<int, int>> inner;   // (slot, binary node)
    for (int k = 0; k < (int)kids.size(); ++k) {
        const BinNode &c = B.nodes[kids[k]];
        n.qlo_x[k] = q_lo(c.box.lo[0], org[0], sc[0]); n.qhi_x[k] = q_hi(c.box.hi[0], org[0], sc[0]);
        n.qlo_y[k] = q_lo(c.box.lo[1], org[1], sc[1]); n.qhi_y[k] = q_hi(c.box.hi[1], org[1], sc[1]);
        n.qlo_z[k] = q_lo(c.box.lo[2], org[2], sc[2]); n.qhi_z[k] = q_hi(c.box.hi[2], org[2], sc[2]);
        if (c.left < 0) { n.child[k] = c.first; n.count[k] = (uint8_t)c.count; }
        else inner.push_back({k, kids[k]});
    }
    for (auto &pr : inner) {
        const int idx = (int)out.size();
        out.emplace_back();
        n.child[pr.first] = idx;
        n.count[pr.first] = 0;
    }
    out[wi] = n;
    for (auto &pr : inner) collapse8(B, pr.second, out, out[wi].child[pr.first]);
}

static void build_binary(Builder &B, const float *tri, int n)
{
    B.tbox.resize(n);
    B.cent.resize(3 * (size_t)n);
    B.ref.resize(n);
    for (int i = 0; i < n; ++i) {
        Box b;
        for (int v = 0; v < 3; ++v) b.grow(tri + 9 * (size_t)i + 3 * v);
        B.tbox[i] = b;
        for (int k = 0; k < 3; ++k) B.cent[3 * (size_t)i + k] = 0.5f * (b.lo[k] + b.hi[k]);
        B.ref[i] = i;
    }
    B.nodes.reserve(2 * (size_t)n + 1);
    B.build(0, n);
}

}  // namespace ptbvh

// Builds the 4-wide BVH and, when nodes8 is given, the 8-wide one over the same leaves.
// tri: n*9 floats. Writes nodes and the triangle order (order[i] = input index of the i-th
// triangle in BVH order).
void pt_build_bvh(const float *tri, int n, std::vector<BNode> &nodes, std::vector<BNode8> *nodes8,
                  std::vector<int> &order)
{
    using namespace ptbvh;
    Builder B;
    build_binary(B, tri, n);
    nodes.clear();
    nodes.emplace_back();
    collapse(B, 0, nodes, 0);
    if (nodes8) {
        nodes8->clear();
        nodes8->emplace_back();
        collapse8(B, 0, *nodes8, 0);
    }
    order = B.ref;
}

void pt_build_bvh4(const float *tri, int n, std::vector<BNode> &nodes, std::vector<int> &order)
{
    pt_build_bvh(tri, n, nodes, nullptr, order);
}

namespace {
void stack_need_rec(const std::vector<BNode> &nodes, int n, int level, int &need, int &depth)
{
    int inner = 0, best = 0, deepest = level;
    for (int k = 0; k < 4; ++k) {
        if (nodes[n].count[k] != 0) continue;
        ++inner;
        int nd = 0, dp = 0;
        stack_need_rec(nodes, nodes[n].child[k], level + 1, nd, dp);
        best = std::max(best, nd);
        deepest = std::max(deepest, dp);
    }
    need = std::max(inner - 1, 0) + best;
    depth = deepest;
}
}  // namespace

// Largest traversal stack a walk of the 4-wide tree can need: at a node with k inner children the
// walk continues into one of them and pushes at most k - 1, so a subtree needs max(k - 1, 0) plus
// the largest need of its inner children. depth receives the number of node levels.
int pt_bvh4_stack_need(const std::vector<BNode> &nodes, int *depth)
{
    int need = 0, dp = 1;
    if (!nodes.empty()) stack_need_rec(nodes, 0, 1, need, dp);
    if (depth) *depth = dp;
    return need;
}

namespace {
void stack_need8_rec(const std::vector<BNode8> &nodes, int n, int level, int &need, int &depth)
{
    int inner = 0, best = 0, deepest = level;
    for (int k = 0; k < 8; ++k) {
        if (nodes[n].count[k] != 0) continue;
        ++inner;
        int nd = 0, dp = 0;
        stack_need8_rec(nodes, nodes[n].child[k], level + 1, nd, dp);
        best = std::max(best, nd);
        deepest = std::max(deepest, dp);
    }
    need = std::max(inner - 1, 0) + best;
    depth = deepest;
}
}  // namespace

// the same bound for the 8-wide tree
int pt_bvh8_stack_need(const std::vector<BNode8> &nodes, int *depth)
{
    int need = 0, dp = 1;
    if (!nodes.empty()) stack_need8_rec(nodes, 0, 1, need, dp);
    if (depth) *depth = dp;
    return need;
}
