// Host BVH builder: binned surface-area-heuristic BVH2 over triangles, laid out for the
// gfx950 traversal kernel (both child boxes stored in the parent, 64 bytes per node).
#include "bvh.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <future>
#include <limits>

namespace nrrs {
namespace {

struct Box {
  float lo[3], hi[3];
  void reset() {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::numeric_limits<float>::infinity();
      hi[k] = -std::numeric_limits<float>::infinity();
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
    if (!(hi[0] >= lo[0])) return 0.0;
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
};

constexpr int kBins = 32;
constexpr uint32_t kLeafMax = kLeafMaxTris;  // (the link encoding would allow 8)
constexpr uint32_t kLeafTarget = 4;
constexpr int kSahDepth = 32;      // beyond this depth, median splits bound the tree depth

struct Builder {
  const std::vector<Box>* tb;
  const std::vector<float>* cen;  // 3 per triangle
  std::vector<uint32_t>* order;
  // nodes are produced as (box0, box1, link0, link1)
  struct Node {
    Box b[2];
    uint32_t link[2];
  };
  std::vector<Node> nodes;

  static uint32_t leaf_link(uint32_t first, uint32_t count) { return 0x80000000u | (first << 3) | (count - 1); }

  // Splits [a, b) and returns the split point, or a == b meaning "make a leaf".
  uint32_t split(uint32_t a, uint32_t b, const Box& bounds, int depth) {
    const uint32_t n = b - a;
    Box cb;
    cb.reset();
    for (uint32_t i = a; i < b; ++i) cb.grow(&(*cen)[3 * (*order)[i]]);
    int axis = 0;
    for (int k = 1; k < 3; ++k)
      if (cb.hi[k] - cb.lo[k] > cb.hi[axis] - cb.lo[axis]) axis = k;
    const float ext = cb.hi[axis] - cb.lo[axis];
    if (!(ext > 0.0f)) {
      if (n <= kLeafMax) return a;
      return a + n / 2;  // identical centroids: split the range in two
    }
    if (depth >= kSahDepth) {
      // depth limit: median split along the longest axis keeps the tree shallow
      uint32_t m = a + n / 2;
      std::nth_element(order->begin() + a, order->begin() + m, order->begin() + b, [&](uint32_t x, uint32_t y) {
        return (*cen)[3 * x + axis] < (*cen)[3 * y + axis];
      });
      return m;
    }
    // binned SAH over all three axes
    double best_cost = std::numeric_limits<double>::infinity();
    int best_axis = -1, best_split = -1;
    for (int ax = 0; ax < 3; ++ax) {
      const float e = cb.hi[ax] - cb.lo[ax];
      if (!(e > 0.0f)) continue;
      const float scale = kBins / e;
      Box bb[kBins];
      uint32_t cnt[kBins] = {0};
      for (int k = 0; k < kBins; ++k) bb[k].reset();
      for (uint32_t i = a; i < b; ++i) {
        const uint32_t t = (*order)[i];
        int bin = std::min(kBins - 1, (int)(((*cen)[3 * t + ax] - cb.lo[ax]) * scale));
        cnt[bin]++;
        bb[bin].grow((*tb)[t]);
      }
      double right_area[kBins];
      uint32_t right_cnt[kBins];
      Box acc;
      acc.reset();
      uint32_t c = 0;
      for (int k = kBins - 1; k > 0; --k) {
        acc.grow(bb[k]);
        c += cnt[k];
        right_area[k] = acc.area();
        right_cnt[k] = c;
      }
      acc.reset();
      c = 0;
      for (int k = 0; k < kBins - 1; ++k) {
        acc.grow(bb[k]);
        c += cnt[k];
        if (c == 0 || right_cnt[k + 1] == 0) continue;
        double cost = acc.area() * c + right_area[k + 1] * right_cnt[k + 1];
        if (cost < best_cost) {
          best_cost = cost;
          best_axis = ax;
          best_split = k;
        }
      }
    }
    const double leaf_cost = bounds.area() * n;
    if (best_axis < 0 || (n <= kLeafTarget) || (n <= kLeafMax && best_cost >= leaf_cost)) {
      if (n <= kLeafMax) return a;
      if (best_axis < 0) return a + n / 2;
    }
    const float e = cb.hi[best_axis] - cb.lo[best_axis];
    const float scale = kBins / e;
    auto mid = std::partition(order->begin() + a, order->begin() + b, [&](uint32_t t) {
      int bin = std::min(kBins - 1, (int)(((*cen)[3 * t + best_axis] - cb.lo[best_axis]) * scale));
      return bin <= best_split;
    });
    uint32_t m = (uint32_t)(mid - order->begin());
    if (m == a || m == b) m = a + n / 2;
    return m;
  }

  Box range_box(uint32_t a, uint32_t b) {
    Box r;
    r.reset();
    for (uint32_t i = a; i < b; ++i) r.grow((*tb)[(*order)[i]]);
    return r;
  }

  int max_depth = 0;

  // Builds the subtree of [a, b) and returns its link (leaf link or node index).
  uint32_t build(uint32_t a, uint32_t b, const Box& bounds, int depth) {
    if (depth > max_depth) max_depth = depth;
    uint32_t m = split(a, b, bounds, depth);
    if (m == a) return leaf_link(a, b - a);
    uint32_t id = (uint32_t)nodes.size();
    nodes.push_back(Node{});
    Box lb = range_box(a, m), rb = range_box(m, b);
    uint32_t l = build(a, m, lb, depth + 1);
    uint32_t r = build(m, b, rb, depth + 1);
    nodes[id].b[0] = lb;
    nodes[id].b[1] = rb;
    nodes[id].link[0] = l;
    nodes[id].link[1] = r;
    return id;
  }
};

}  // namespace

namespace {

// The tree over items with boxes tb and centroids cen (3 per item).
void build_tree(const std::vector<Box>& tb, const std::vector<float>& cen, uint64_t nt, BvhOut& out, bool wide);

}  // namespace

int build_bvh(const float* verts, const uint32_t* tris, uint64_t nt, BvhOut& out, bool wide) {
  std::vector<Box> tb(nt);
  std::vector<float> cen(3 * nt);
  for (uint64_t i = 0; i < nt; ++i) {
    tb[i].reset();
    for (int c = 0; c < 3; ++c) tb[i].grow(verts + 3 * (uint64_t)tris[3 * i + c]);
    for (int k = 0; k < 3; ++k) cen[3 * i + k] = 0.5f * (tb[i].lo[k] + tb[i].hi[k]);
  }
  build_tree(tb, cen, nt, out, wide);
  return 0;
}

int build_bvh_boxes(const float* boxes, uint64_t n, BvhOut& out) {
  std::vector<Box> tb(n);
  std::vector<float> cen(3 * n);
  for (uint64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) {
      tb[i].lo[k] = boxes[6 * i + k];
      tb[i].hi[k] = boxes[6 * i + 3 + k];
      cen[3 * i + k] = 0.5f * (tb[i].lo[k] + tb[i].hi[k]);
    }
  }
  build_tree(tb, cen, n, out, false);
  return 0;
}

namespace {

void build_tree(const std::vector<Box>& tb, const std::vector<float>& cen, uint64_t nt, BvhOut& out, bool wide) {
  out.order.resize(nt);
  for (uint64_t i = 0; i < nt; ++i) out.order[i] = (uint32_t)i;
  Builder B{&tb, &cen, &out.order, {}};
  B.nodes.reserve(nt > 0 ? 2 * nt / kLeafTarget + 16 : 16);
  // The root is always an internal node so traversal starts by testing two child boxes.
  Box all = B.range_box(0, (uint32_t)nt);
  uint32_t root_link = B.build(0, (uint32_t)nt, all, 0);
  if (root_link & 0x80000000u) {
    Builder::Node r{};
    r.b[0] = all;
    // The second child repeats triangle 0 behind an inverted box.  Slab tests order each
    // axis's two distances, so rays may still enter it; testing triangle 0 twice leaves the
    // closest hit unchanged (same distance, same index).
    r.b[1].reset();
    r.link[0] = root_link;
    r.link[1] = Builder::leaf_link(0, 1);
    B.nodes.insert(B.nodes.begin(), r);
  }
  out.n_nodes = B.nodes.size();
  out.max_depth = B.max_depth + 1;
  out.nodes.resize(16 * out.n_nodes);
  for (size_t i = 0; i < B.nodes.size(); ++i) {
    const auto& n = B.nodes[i];
    float* f = &out.nodes[16 * i];
    f[0] = n.b[0].lo[0]; f[1] = n.b[0].lo[1]; f[2] = n.b[0].lo[2]; f[3] = n.b[0].hi[0];
    f[4] = n.b[0].hi[1]; f[5] = n.b[0].hi[2]; f[6] = n.b[1].lo[0]; f[7] = n.b[1].lo[1];
    f[8] = n.b[1].lo[2]; f[9] = n.b[1].hi[0]; f[10] = n.b[1].hi[1]; f[11] = n.b[1].hi[2];
    std::memcpy(&f[12], &n.link[0], 4);
    std::memcpy(&f[13], &n.link[1], 4);
    f[14] = 0.0f;
    f[15] = 0.0f;
  }
  if (wide) collapse_bvh4(out);
}

}  // namespace

namespace {

struct Child4 {
  float lo[3], hi[3];
  uint32_t link;  // BVH2 leaf link, or a BVH2 node index while collapsing
  double area() const {
    const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return dx >= 0.0 ? 2.0 * (dx * dy + dy * dz + dz * dx) : 0.0;
  }
};

struct Collapser {
  const std::vector<float>* n2;
  std::vector<float>* n4;
  int max_depth = 0;

  Child4 child_of(uint32_t node2, int c) const {
    const float* f = &(*n2)[16ull * node2];
    Child4 ch;
    for (int k = 0; k < 3; ++k) {
      ch.lo[k] = f[6 * c + k];
      ch.hi[k] = f[6 * c + 3 + k];
    }
    std::memcpy(&ch.link, &f[12 + c], 4);
    return ch;
  }

  // Builds the 4-wide node for BVH2 node `node2`; returns its index.
  uint32_t build(uint32_t node2, int depth) {
    if (depth > max_depth) max_depth = depth;
    Child4 ch[4];
    int m = 2;
    ch[0] = child_of(node2, 0);
    ch[1] = child_of(node2, 1);
    while (m < 4) {
      int best = -1;
      double best_area = -1.0;
      for (int k = 0; k < m; ++k)
        if (!(ch[k].link & 0x80000000u) && ch[k].area() > best_area) {
          best_area = ch[k].area();
          best = k;
        }
      if (best < 0) break;
      const uint32_t open = ch[best].link;
      ch[best] = child_of(open, 0);
      ch[m++] = child_of(open, 1);
    }
    const uint32_t id = (uint32_t)(n4->size() / 32);
    n4->resize(n4->size() + 32, 0.0f);
    uint32_t links[4];
    for (int k = 0; k < 4; ++k) {
      if (k >= m) {
        links[k] = kEmptyChild4;
        continue;
      }
      links[k] = (ch[k].link & 0x80000000u) ? ch[k].link : build(ch[k].link, depth + 1);
    }
    float* f = &(*n4)[32ull * id];
    for (int k = 0; k < 4; ++k) {
      const bool used = k < m;
      for (int a = 0; a < 3; ++a) {
        f[8 * a + k] = used ? ch[k].lo[a] : 0.0f;      // lo of axis a
        f[8 * a + 4 + k] = used ? ch[k].hi[a] : 0.0f;  // hi of axis a
      }
      std::memcpy(&f[24 + k], &links[k], 4);
      f[28 + k] = 0.0f;
    }
    return id;
  }
};

}  // namespace

void collapse_bvh4(BvhOut& out) {
  out.nodes4.clear();
  out.nodes4.reserve(out.nodes.size());
  Collapser c{&out.nodes, &out.nodes4};
  c.build(0, 0);
  out.n_nodes4 = out.nodes4.size() / 32;
  out.max_depth4 = c.max_depth + 1;
}

}  // namespace nrrs
