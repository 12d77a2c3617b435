// Scene validation, per-instance records and the BVH over instance AABBs.
//
// Paper correspondence: a geometry is an AABB plus instances (Sec. 3.1
// "BLAS from Geometry"; Sec. 4.1, listing "Procedural geometry creation");
// the acceleration structure is one BLAS per geometry and one TLAS over all
// instances, whose sequential instance index is its creation order (Sec.
// 3.1); the transforms live in an instance buffer so that intersection works
// in local space (listing "Instance buffer creation").  Here a geometry's
// BLAS is its single AABB, so the structure reduces to one binned-SAH BVH
// over the instances' world-space AABBs; leaf order reorders the 128-byte
// instance records so that a leaf's instances are contiguous.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <numeric>

#include "host_common.h"

using namespace pr;

namespace pr {

static thread_local std::string g_err;

pr_status set_error(pr_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

pr_status ok() {
  g_err.clear();
  return PR_OK;
}

pr_status hip_fail(hipError_t e, const char* what) {
  return set_error(PR_ERR_DEVICE, "%s failed: %s", what, hipGetErrorString(e));
}

}  // namespace pr

namespace {

constexpr uint32_t kMaxInstances = 16384;   // BVH stack entries (node, child) fit 16 bits
constexpr int kMaxDepth = 30;               // traversal stack holds depth + 2 entries

bool finite3(const float* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// inverse of a 3x3 (row-major) in double; returns determinant
double inv3(const double A[9], double out[9]) {
  double c00 = A[4] * A[8] - A[5] * A[7];
  double c01 = A[5] * A[6] - A[3] * A[8];
  double c02 = A[3] * A[7] - A[4] * A[6];
  double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  if (det == 0.0) return 0.0;
  double id = 1.0 / det;
  out[0] = c00 * id;
  out[1] = (A[2] * A[7] - A[1] * A[8]) * id;
  out[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  out[3] = c01 * id;
  out[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  out[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  out[6] = c02 * id;
  out[7] = (A[1] * A[6] - A[0] * A[7]) * id;
  out[8] = (A[0] * A[4] - A[1] * A[3]) * id;
  return det;
}

// smallest singular value of A: sqrt of the smallest eigenvalue of A^T A
// (cyclic Jacobi on the symmetric 3x3)
double sigma_min(const double A[9]) {
  double S[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[k * 3 + i] * A[k * 3 + j];
      S[i][j] = s;
    }
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = S[0][1] * S[0][1] + S[0][2] * S[0][2] + S[1][2] * S[1][2];
    if (off < 1e-30 * (S[0][0] * S[0][0] + S[1][1] * S[1][1] + S[2][2] * S[2][2])) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (S[p][q] == 0.0) continue;
        double theta = (S[q][q] - S[p][p]) / (2.0 * S[p][q]);
        double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < 3; ++k) {
          double skp = S[k][p], skq = S[k][q];
          S[k][p] = c * skp - s * skq;
          S[k][q] = s * skp + c * skq;
        }
        for (int k = 0; k < 3; ++k) {
          double spk = S[p][k], sqk = S[q][k];
          S[p][k] = c * spk - s * sqk;
          S[q][k] = s * spk + c * sqk;
        }
      }
  }
  double ev = std::min(S[0][0], std::min(S[1][1], S[2][2]));
  return std::sqrt(std::max(ev, 0.0));
}

pr_status pack_params(const pr_geometry& g, float out[8]) {
  const float* p = g.params;
  for (int i = 0; i < 8; ++i) out[i] = 0.f;
  if (!finite3(p, 8)) return set_error(PR_ERR_INVALID_ARG, "non-finite geometry parameter");
  switch (g.type) {
    case PR_SPHERE:
      if (!(p[0] > 0)) return set_error(PR_ERR_INVALID_ARG, "sphere radius must be > 0");
      out[0] = p[0];
      break;
    case PR_BOX:
      if (!(p[3] > 0 && p[4] > 0 && p[5] > 0))
        return set_error(PR_ERR_INVALID_ARG, "box half extents must be > 0");
      for (int i = 0; i < 6; ++i) out[i] = p[i];
      break;
    case PR_TORUS:
      if (!(p[0] > 0 && p[1] > 0)) return set_error(PR_ERR_INVALID_ARG, "torus radii must be > 0");
      out[0] = p[0];
      out[1] = p[1];
      break;
    case PR_BOXFRAME:
      if (!(p[0] > 0 && p[1] > 0 && p[1] < p[0]))
        return set_error(PR_ERR_INVALID_ARG, "box-frame needs 0 < e < b");
      out[0] = p[0];
      out[1] = p[1];
      out[2] = p[0] - p[1];
      break;
    case PR_PACMAN:
      if (!(p[0] > 0 && p[1] > 0 && p[1] < 1.5707963f))
        return set_error(PR_ERR_INVALID_ARG, "pac-man needs R > 0 and 0 < alpha < pi/2");
      out[0] = p[0];
      out[1] = (float)std::cos((double)p[1]);
      out[2] = (float)std::sin((double)p[1]);
      break;
    case PR_JULIA: {
      const double nit = p[4], bail = p[5];
      if (!(nit >= 1 && nit <= 64 && nit == std::floor(nit)))
        return set_error(PR_ERR_INVALID_ARG, "julia n_iter must be an integer in 1..64");
      if (!(bail > 0)) return set_error(PR_ERR_INVALID_ARG, "julia bailout must be > 0");
      // m^2 <= (2 bailout)^(2 n_iter) must stay finite in float32
      if (2.0 * nit * std::log2(std::max(2.0 * bail, 1.0)) > 120.0)
        return set_error(PR_ERR_UNSUPPORTED,
                         "julia n_iter * log2(2 bailout) > 60 overflows the float32 derivative");
      for (int i = 0; i < 4; ++i) out[i] = p[i];
      out[4] = p[4];
      out[5] = (float)(bail * bail);
      break;
    }
    case PR_MANDELBULB: {
      const double power = p[0], nit = p[1], bail = p[2];
      if (!(nit >= 1 && nit <= 64 && nit == std::floor(nit)))
        return set_error(PR_ERR_INVALID_ARG, "mandelbulb n_iter must be an integer in 1..64");
      if (!(bail > 0)) return set_error(PR_ERR_INVALID_ARG, "mandelbulb bailout must be > 0");
      if (!(power >= 2)) return set_error(PR_ERR_INVALID_ARG, "mandelbulb power must be >= 2");
      if (power != 8.0) return set_error(PR_ERR_UNSUPPORTED, "only the power-8 Mandelbulb is implemented");
      if (nit * std::log2(std::max(8.0 * std::pow(bail, 7.0), 1.0)) > 120.0)
        return set_error(PR_ERR_UNSUPPORTED,
                         "mandelbulb n_iter * log2(8 bailout^7) > 120 overflows the float32 derivative");
      out[0] = p[1];
      out[1] = (float)(bail * bail);
      break;
    }
    default:
      if (user_type_registered(g.type)) {
        // user estimator: parameters are passed through as given
        for (int i = 0; i < 7; ++i) out[i] = p[i];
        break;
      }
      return set_error(PR_ERR_INVALID_ARG, "unknown primitive type %u", g.type);
  }
  return PR_OK;
}

// ------------------------------------------------------------------ BVH
struct Box {
  double lo[3], hi[3];
  void empty() {
    for (int i = 0; i < 3; ++i) {
      lo[i] = std::numeric_limits<double>::infinity();
      hi[i] = -std::numeric_limits<double>::infinity();
    }
  }
  void grow(const Box& b) {
    for (int i = 0; i < 3; ++i) {
      lo[i] = std::min(lo[i], b.lo[i]);
      hi[i] = std::max(hi[i], b.hi[i]);
    }
  }
  double area() const {
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    if (dx < 0 || dy < 0 || dz < 0) return 0.0;
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
};

struct BuildItem {
  uint32_t node, begin, end;
  int depth;
};

void build_bvh(pr_scene* s, const pr_bvh_opts& o) {
  const uint32_t n = (uint32_t)s->host_insts.size();
  std::vector<Box> boxes(n);
  std::vector<double> cen(3 * n);
  for (uint32_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) {
      boxes[i].lo[a] = s->world_aabb[6 * i + a];
      boxes[i].hi[a] = s->world_aabb[6 * i + 3 + a];
      cen[3 * i + a] = 0.5 * (boxes[i].lo[a] + boxes[i].hi[a]);
    }
  }
  std::vector<uint32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0u);
  std::vector<HostNode> nodes;
  nodes.reserve(2 * n);
  nodes.push_back(HostNode{});
  std::deque<BuildItem> work;   // breadth-first: top levels get the lowest indices
  work.push_back({0, 0, n, 0});
  const uint32_t bins = o.sah_bins;
  std::vector<Box> bin_box(bins);
  std::vector<uint32_t> bin_cnt(bins);
  auto finish_node = [&](uint32_t ni, const Box& b) {
    // inflate so that float32 slab tests never cull what the exact local
    // test would accept
    for (int a = 0; a < 3; ++a) {
      double ext = b.hi[a] - b.lo[a];
      double pad = 1e-5 * std::max(ext, 1.0) + 1e-6 * std::max(std::fabs(b.lo[a]), std::fabs(b.hi[a]));
      nodes[ni].lo[a] = std::nextafter((float)(b.lo[a] - pad), -INFINITY);
      nodes[ni].hi[a] = std::nextafter((float)(b.hi[a] + pad), INFINITY);
    }
  };
  while (!work.empty()) {
    BuildItem it = work.front();
    work.pop_front();
    Box nb, cb;
    nb.empty();
    cb.empty();
    for (uint32_t k = it.begin; k < it.end; ++k) {
      nb.grow(boxes[idx[k]]);
      Box c;
      for (int a = 0; a < 3; ++a) c.lo[a] = c.hi[a] = cen[3 * idx[k] + a];
      cb.grow(c);
    }
    finish_node(it.node, nb);
    const uint32_t cnt = it.end - it.begin;
    if (cnt <= o.max_leaf) {
      nodes[it.node].first = it.begin;
      nodes[it.node].count = cnt;
      continue;
    }
    // choose a split: binned SAH while shallow, median split near the depth limit
    int best_axis = -1;
    uint32_t best_bin = 0;
    double best_cost = std::numeric_limits<double>::infinity();
    const bool sah = it.depth < kMaxDepth - 16;
    if (sah) {
      for (int a = 0; a < 3; ++a) {
        double ext = cb.hi[a] - cb.lo[a];
        if (!(ext > 0)) continue;
        for (uint32_t b = 0; b < bins; ++b) {
          bin_box[b].empty();
          bin_cnt[b] = 0;
        }
        for (uint32_t k = it.begin; k < it.end; ++k) {
          uint32_t b = (uint32_t)std::min<double>(bins - 1, (cen[3 * idx[k] + a] - cb.lo[a]) / ext * bins);
          bin_box[b].grow(boxes[idx[k]]);
          ++bin_cnt[b];
        }
        std::vector<double> right_area(bins), right_cnt(bins);
        Box acc;
        acc.empty();
        uint32_t c = 0;
        for (int b = (int)bins - 1; b > 0; --b) {
          acc.grow(bin_box[b]);
          c += bin_cnt[b];
          right_area[b] = acc.area();
          right_cnt[b] = c;
        }
        acc.empty();
        c = 0;
        for (uint32_t b = 0; b + 1 < bins; ++b) {
          acc.grow(bin_box[b]);
          c += bin_cnt[b];
          if (c == 0 || right_cnt[b + 1] == 0) continue;
          double cost = o.c_node + (acc.area() * c + right_area[b + 1] * right_cnt[b + 1]) *
                                       o.c_leaf / std::max(nb.area(), 1e-300);
          if (cost < best_cost) {
            best_cost = cost;
            best_axis = a;
            best_bin = b;
          }
        }
      }
    }
    uint32_t mid;
    if (best_axis >= 0) {
      const int a = best_axis;
      const double ext = cb.hi[a] - cb.lo[a];
      auto pmid = std::partition(idx.begin() + it.begin, idx.begin() + it.end, [&](uint32_t i) {
        uint32_t b = (uint32_t)std::min<double>(bins - 1, (cen[3 * i + a] - cb.lo[a]) / ext * bins);
        return b <= best_bin;
      });
      mid = (uint32_t)(pmid - idx.begin());
    } else {
      // median split along the widest centroid axis (or by index when all coincide)
      int a = 0;
      for (int k = 1; k < 3; ++k)
        if (cb.hi[k] - cb.lo[k] > cb.hi[a] - cb.lo[a]) a = k;
      mid = it.begin + cnt / 2;
      std::nth_element(idx.begin() + it.begin, idx.begin() + mid, idx.begin() + it.end,
                       [&](uint32_t x, uint32_t y) {
                         return cen[3 * x + a] < cen[3 * y + a] || (cen[3 * x + a] == cen[3 * y + a] && x < y);
                       });
    }
    if (mid == it.begin || mid == it.end) mid = it.begin + cnt / 2;
    const uint32_t left = (uint32_t)nodes.size();
    nodes.push_back(HostNode{});
    nodes.push_back(HostNode{});
    nodes[it.node].first = left;
    nodes[it.node].count = 0;
    work.push_back({left, it.begin, mid, it.depth + 1});
    work.push_back({left + 1, mid, it.end, it.depth + 1});
  }
  s->nodes = std::move(nodes);
  s->order = std::move(idx);
  // device layout: one record per interior node (breadth-first order kept),
  // each holding both children's boxes and references
  const std::vector<HostNode>& hn = s->nodes;
  std::vector<uint32_t> dev_index(hn.size(), kNoChild);
  uint32_t n_int = 0;
  for (size_t i = 0; i < hn.size(); ++i)
    if (hn[i].count == 0) dev_index[i] = n_int++;
  std::vector<NodeDev> dn(std::max<uint32_t>(n_int, 1));
  auto fill_child = [&](float* lo, float* hi, uint32_t& c, uint32_t& cnt, uint32_t h) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = hn[h].lo[a];
      hi[a] = hn[h].hi[a];
    }
    if (hn[h].count == 0) {
      c = dev_index[h];
      cnt = 0;
    } else {
      c = hn[h].first;
      cnt = hn[h].count;
    }
  };
  if (n_int == 0) {
    // a single leaf: the root record has that leaf as its only child
    NodeDev& d = dn[0];
    fill_child(d.lo0, d.hi0, d.c0, d.n0, 0);
    for (int a = 0; a < 3; ++a) {
      d.lo1[a] = 0.f;
      d.hi1[a] = 0.f;
    }
    d.c1 = 0;
    d.n1 = kNoChild;
  } else {
    for (size_t i = 0; i < hn.size(); ++i) {
      if (hn[i].count != 0) continue;
      NodeDev& d = dn[dev_index[i]];
      fill_child(d.lo0, d.hi0, d.c0, d.n0, hn[i].first);
      fill_child(d.lo1, d.hi1, d.c1, d.n1, hn[i].first + 1);
    }
  }
  s->dnodes = std::move(dn);
}

// The four-wide device BVH: each node takes the two children of a host
// interior node and, while it has fewer than four, replaces its interior
// child of largest surface area by that child's two children.  Nodes are
// numbered breadth first (the top levels are the ones staged in LDS).
// Leaves s->dnodes4 empty when the tree would not fit the kernel's limits
// (node indices, the traversal stack in the worst case, leaf encoding) or a
// quantized box could not be made to contain its child.
void build_bvh4(pr_scene* s) {
  s->dnodes4.clear();
  const std::vector<HostNode>& hn = s->nodes;
  if (hn.empty()) return;
  auto area = [&](uint32_t h) {
    const double dx = (double)hn[h].hi[0] - hn[h].lo[0], dy = (double)hn[h].hi[1] - hn[h].lo[1],
                 dz = (double)hn[h].hi[2] - hn[h].lo[2];
    return dx * dy + dy * dz + dz * dx;
  };
  std::vector<uint32_t> queue{0};   // host node of each four-wide node, breadth first
  std::vector<Node4Dev> out;
  for (size_t i = 0; i < queue.size(); ++i) {
    const uint32_t h = queue[i];
    std::vector<uint32_t> c;
    if (hn[h].count != 0) {
      c.push_back(h);   // a single-leaf tree: the root node holds that leaf
    } else {
      c = {hn[h].first, hn[h].first + 1};
      while (c.size() < 4) {
        int best = -1;
        for (size_t k = 0; k < c.size(); ++k)
          if (hn[c[k]].count == 0 && (best < 0 || area(c[k]) > area(c[best]))) best = (int)k;
        if (best < 0) break;
        const uint32_t x = c[best];
        c[best] = hn[x].first;
        c.insert(c.begin() + best + 1, hn[x].first + 1);
      }
    }
    Node4Dev d{};
    float plo[3], phi[3];
    for (int a = 0; a < 3; ++a) {
      plo[a] = hn[c[0]].lo[a];
      phi[a] = hn[c[0]].hi[a];
      for (uint32_t x : c) {
        plo[a] = std::min(plo[a], hn[x].lo[a]);
        phi[a] = std::max(phi[a], hn[x].hi[a]);
      }
      // cells of at least 2^-20 of the coordinates' magnitude, so that one
      // cell exceeds the float32 rounding of a decoded bound
      const float mag = std::max({std::fabs(plo[a]), std::fabs(phi[a]), 1e-30f});
      float step = std::max((phi[a] - plo[a]) / 253.0f, mag * 9.5367431640625e-7f);
      d.step[a] = step;
      d.org[a] = plo[a] - step;
    }
    uint32_t refs[4] = {kNoRef, kNoRef, kNoRef, kNoRef};
    for (size_t k = 0; k < c.size(); ++k) {
      const HostNode& x = hn[c[k]];
      for (int a = 0; a < 3; ++a) {
        double ql = std::floor(((double)x.lo[a] - d.org[a]) / d.step[a]) - 1.0;
        double qh = std::ceil(((double)x.hi[a] - d.org[a]) / d.step[a]) + 1.0;
        int lo = (int)std::min(255.0, std::max(0.0, ql)), hi = (int)std::min(255.0, std::max(0.0, qh));
        // the kernel decodes org + q * step in float32: make sure the box
        // contains the child's
        while (lo > 0 && std::fmaf((float)lo, d.step[a], d.org[a]) > x.lo[a]) --lo;
        while (hi < 255 && std::fmaf((float)hi, d.step[a], d.org[a]) < x.hi[a]) ++hi;
        if (std::fmaf((float)lo, d.step[a], d.org[a]) > x.lo[a] || std::fmaf((float)hi, d.step[a], d.org[a]) < x.hi[a])
          return;
        d.q[6 * k + a] = (uint8_t)lo;
        d.q[6 * k + 3 + a] = (uint8_t)hi;
      }
      if (x.count != 0) {
        if (x.count > 128 || x.first >= (1u << 24)) return;
        refs[k] = (1u << 31) | ((x.count - 1) << 24) | x.first;
      } else {
        refs[k] = (uint32_t)queue.size();
        queue.push_back(c[k]);
      }
    }
    d.ref0 = refs[0];
    d.ref1 = refs[1];
    d.ref2 = refs[2];
    d.ref3 = refs[3];
    out.push_back(d);
    if (queue.size() > kMaxNodes4) return;
  }
  // worst-case stack use: descending into one child pushes its hit siblings
  std::vector<int> need(out.size(), 0);
  for (size_t i = out.size(); i-- > 0;) {
    const uint32_t r[4] = {out[i].ref0, out[i].ref1, out[i].ref2, out[i].ref3};
    int n = 0, deepest = 0;
    for (uint32_t x : r)
      if (x != kNoRef) {
        ++n;
        if (!(x >> 31)) deepest = std::max(deepest, need[x]);
      }
    need[i] = (n - 1) + deepest;
  }
  if (need[0] + 1 > kStackDepth) return;
  // every instance slot in exactly one leaf, every child index in range
  std::vector<uint8_t> seen(s->order.size(), 0);
  for (const Node4Dev& d : out) {
    const uint32_t r[4] = {d.ref0, d.ref1, d.ref2, d.ref3};
    for (uint32_t x : r) {
      if (x == kNoRef) continue;
      if (x >> 31) {
        const uint32_t first = x & 0xffffffu, n = ((x >> 24) & 0x7fu) + 1;
        for (uint32_t k = first; k < first + n; ++k) {
          if (k >= seen.size() || seen[k]) return;
          seen[k] = 1;
        }
      } else if (x == 0 || x >= out.size()) {
        return;
      }
    }
  }
  for (uint8_t v : seen)
    if (!v) return;
  s->dnodes4 = std::move(out);
}

int bvh_depth(const std::vector<HostNode>& nodes, uint32_t ni) {
  if (nodes[ni].count > 0) return 0;
  return 1 + std::max(bvh_depth(nodes, nodes[ni].first), bvh_depth(nodes, nodes[ni].first + 1));
}

}  // namespace

// C ABI struct layouts (the Python binding asserts the same sizes)
static_assert(sizeof(pr_geometry) == 76, "pr_geometry layout");
static_assert(sizeof(pr_instance) == 56, "pr_instance layout");
static_assert(sizeof(pr_material) == 16, "pr_material layout");
static_assert(sizeof(pr_scene_consts) == 40, "pr_scene_consts layout");
static_assert(sizeof(pr_camera) == 40, "pr_camera layout");
static_assert(sizeof(pr_render_opts) == 72, "pr_render_opts layout");
static_assert(sizeof(pr_batch_opts) == 20, "pr_batch_opts layout");

extern "C" {

uint32_t pr_abi_version(void) { return PR_ABI_VERSION; }

const char* pr_last_error(void) { return g_err.c_str(); }

uint32_t pr_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return (uint32_t)std::max(n, 0);
}

pr_status pr_scene_create(const pr_geometry* geoms, uint32_t n_geom, const pr_instance* insts,
                          uint32_t n_inst, const pr_material* mats, uint32_t n_mat,
                          const pr_scene_consts* consts, pr_scene** out) {
  try {
    if (!out) return set_error(PR_ERR_INVALID_ARG, "out is NULL");
    if (!geoms || !insts || !mats || !consts)
      return set_error(PR_ERR_INVALID_ARG, "geoms, insts, mats and consts must be non-NULL");
    if (n_geom == 0 || n_mat == 0) return set_error(PR_ERR_INVALID_ARG, "n_geom and n_mat must be >= 1");
    if (n_inst == 0 || n_inst > kMaxInstances)
      return set_error(PR_ERR_INVALID_ARG, "n_inst must be in 1..%u", kMaxInstances);
    if (!finite3(consts->light_pos, 3) || !finite3(consts->light_rgb, 3) ||
        !std::isfinite(consts->ambient) || !finite3(consts->background, 3))
      return set_error(PR_ERR_INVALID_ARG, "non-finite scene constants");
    std::vector<float> packed(8 * (size_t)n_geom), cuts(4 * (size_t)n_geom);
    for (uint32_t g = 0; g < n_geom; ++g) {
      const pr_aabb& b = geoms[g].aabb;
      if (!finite3(b.lo, 3) || !finite3(b.hi, 3))
        return set_error(PR_ERR_INVALID_ARG, "geometry %u: non-finite AABB", g);
      for (int a = 0; a < 3; ++a)
        if (!(b.lo[a] <= b.hi[a])) return set_error(PR_ERR_INVALID_ARG, "geometry %u: AABB lo > hi", g);
      pr_status st = pack_params(geoms[g], &packed[8 * g]);
      if (st != PR_OK) {
        std::string m = "geometry " + std::to_string(g) + ": " + pr_last_error();
        return set_error(st, "%s", m.c_str());
      }
      // cutting plane (Fig. 5): keep n.p <= d, n normalised here
      const float* c = geoms[g].cut;
      if (!finite3(c, 4)) return set_error(PR_ERR_INVALID_ARG, "geometry %u: non-finite cutting plane", g);
      const double nn = std::sqrt((double)c[0] * c[0] + (double)c[1] * c[1] + (double)c[2] * c[2]);
      if (nn == 0.0) {
        for (int k = 0; k < 4; ++k) cuts[4 * g + k] = 0.f;
      } else if (!(nn > 1e-12)) {
        return set_error(PR_ERR_INVALID_ARG, "geometry %u: cutting-plane normal too small", g);
      } else {
        for (int k = 0; k < 4; ++k) cuts[4 * g + k] = (float)((double)c[k] / nn);
      }
    }
    for (uint32_t m = 0; m < n_mat; ++m) {
      if (!finite3(mats[m].albedo, 3) || !std::isfinite(mats[m].reflectivity) ||
          mats[m].reflectivity < 0.f || mats[m].reflectivity > 1.f)
        return set_error(PR_ERR_INVALID_ARG, "material %u: albedo finite and 0 <= rho <= 1 required", m);
    }
    // Every built-in colour is albedo * (ambient + V lambert light_rgb) with
    // V lambert in [0, 1], the background, or a convex blend of these, so
    // bounding these terms bounds every sample colour (multi-sample means are
    // exact fixed-point sums that need the bound).
    for (int c = 0; c < 3; ++c)
      if (!(std::fabs((double)consts->background[c]) <= (double)kMaxColour))
        return set_error(PR_ERR_INVALID_ARG, "background colour beyond +-2^24");
    for (uint32_t m = 0; m < n_mat; ++m)
      for (int c = 0; c < 3; ++c) {
        const double bound = std::fabs((double)mats[m].albedo[c]) *
                             (std::fabs((double)consts->ambient) + std::fabs((double)consts->light_rgb[c]));
        if (!(bound <= (double)kMaxColour))
          return set_error(PR_ERR_INVALID_ARG,
                           "material %u: |albedo| (|ambient| + |light_rgb|) beyond 2^24 in channel %d", m, c);
      }
    auto* s = new pr_scene();
    s->host_insts.resize(n_inst);
    s->host_shade.resize(4 * (size_t)n_inst);
    s->world_aabb.resize(6 * (size_t)n_inst);
    for (uint32_t i = 0; i < n_inst; ++i) {
      const pr_instance& in = insts[i];
      if (in.geometry >= n_geom || in.material >= n_mat) {
        delete s;
        return set_error(PR_ERR_INVALID_ARG, "instance %u: geometry or material index out of range", i);
      }
      if (!finite3(in.xform, 12)) {
        delete s;
        return set_error(PR_ERR_INVALID_ARG, "instance %u: non-finite transform", i);
      }
      double A[9], Ai[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) A[3 * r + c] = in.xform[4 * r + c];
      double det = inv3(A, Ai);
      if (!(std::fabs(det) > 1e-12)) {
        delete s;
        return set_error(PR_ERR_INVALID_ARG, "instance %u: |det A| <= 1e-12", i);
      }
      const pr_geometry& g = geoms[in.geometry];
      InstDev& d = s->host_insts[i];
      for (int k = 0; k < 9; ++k) d.Ainv[k] = (float)Ai[k];
      for (int r = 0; r < 3; ++r) d.b[r] = in.xform[4 * r + 3];
      for (int a = 0; a < 3; ++a) {
        d.lo[a] = g.aabb.lo[a];
        d.hi[a] = g.aabb.hi[a];
      }
      d.sigma = (float)sigma_min(A);
      d.type = g.type;
      for (int k = 0; k < 8; ++k) d.prm[k] = packed[8 * in.geometry + k];
      uint32_t uid = i;
      std::memcpy(&d.prm[7], &uid, 4);
      for (int k = 0; k < 4; ++k) d.cut[k] = cuts[4 * in.geometry + k];
      for (int k = 0; k < 3; ++k) s->host_shade[4 * (size_t)i + k] = mats[in.material].albedo[k];
      s->host_shade[4 * (size_t)i + 3] = mats[in.material].reflectivity;
      s->n_types_present |= 1u << g.type;
      // world AABB: bounds of the 8 transformed corners (double)
      double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int c = 0; c < 8; ++c) {
        double p[3] = {(c & 1) ? g.aabb.hi[0] : g.aabb.lo[0], (c & 2) ? g.aabb.hi[1] : g.aabb.lo[1],
                       (c & 4) ? g.aabb.hi[2] : g.aabb.lo[2]};
        for (int r = 0; r < 3; ++r) {
          double w = A[3 * r] * p[0] + A[3 * r + 1] * p[1] + A[3 * r + 2] * p[2] + in.xform[4 * r + 3];
          lo[r] = std::min(lo[r], w);
          hi[r] = std::max(hi[r], w);
        }
      }
      for (int r = 0; r < 3; ++r) {
        s->world_aabb[6 * i + r] = (float)lo[r];
        s->world_aabb[6 * i + 3 + r] = (float)hi[r];
      }
    }
    for (int k = 0; k < 3; ++k) {
      s->consts.light[k] = consts->light_pos[k];
      s->consts.light_rgb[k] = consts->light_rgb[k];
      s->consts.background[k] = consts->background[k];
    }
    s->consts.ambient = consts->ambient;
    s->consts.n_inst = n_inst;
    s->n_proc = n_inst;
    s->mats.assign(mats, mats + n_mat);
    *out = s;
    return ok();
  } catch (const std::bad_alloc&) {
    return set_error(PR_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return set_error(PR_ERR_DEVICE, "unexpected exception");
  }
}

static bool scene_busy(pr_scene* s) {
  if (!s->last_use) return false;
  return hipEventQuery(s->last_use) == hipErrorNotReady;
}

static void free_device(pr_scene* s) {
  if (s->d_insts) (void)hipFree(s->d_insts);
  if (s->d_nodes) (void)hipFree(s->d_nodes);
  if (s->d_nodes4) (void)hipFree(s->d_nodes4);
  if (s->d_consts) (void)hipFree(s->d_consts);
  if (s->d_shade) (void)hipFree(s->d_shade);
  s->d_insts = nullptr;
  s->d_nodes = nullptr;
  s->d_nodes4 = nullptr;
  s->d_consts = nullptr;
  s->d_shade = nullptr;
  s->consts.shade = nullptr;
  s->consts.nodes4 = nullptr;
  s->uploaded = false;
  s->device_bytes = 0;
}

pr_status pr_bvh_build(pr_scene* s, const pr_bvh_opts* opts) {
  try {
    if (!s) return set_error(PR_ERR_INVALID_ARG, "scene is NULL");
    pr_bvh_opts o{32, 1, 1.0f, 4.0f, 0};
    if (opts) o = *opts;
    if (o.sah_bins < 4 || o.sah_bins > 256) return set_error(PR_ERR_INVALID_ARG, "sah_bins must be in 4..256");
    if (o.max_leaf < 1 || o.max_leaf > 8) return set_error(PR_ERR_INVALID_ARG, "max_leaf must be in 1..8");
    if (!(o.c_node > 0) || !(o.c_leaf > 0)) return set_error(PR_ERR_INVALID_ARG, "costs must be > 0");
    std::lock_guard<std::mutex> lk(s->mu);
    if (scene_busy(s)) return set_error(PR_ERR_BUSY, "renders of this scene are in flight");
    build_bvh(s, o);
    if (bvh_depth(s->nodes, 0) > kMaxDepth)
      return set_error(PR_ERR_UNSUPPORTED, "BVH deeper than %d levels", kMaxDepth);
    build_bvh4(s);
    s->consts.n_nodes = (uint32_t)s->dnodes.size();
    s->built = true;
    if (o.flags & PR_BVH_HOST_ONLY) return ok();
    free_device(s);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::vector<InstDev> leaf(s->order.size());
    std::vector<float> leaf_shade(4 * s->order.size());
    for (size_t k = 0; k < s->order.size(); ++k) {
      leaf[k] = s->host_insts[s->order[k]];
      for (int c = 0; c < 4; ++c) leaf_shade[4 * k + c] = s->host_shade[4 * (size_t)s->order[k] + c];
    }
    const size_t bi = leaf.size() * sizeof(InstDev), bn = s->dnodes.size() * sizeof(NodeDev);
    const size_t bs = leaf_shade.size() * sizeof(float);
    if ((e = hipMalloc((void**)&s->d_insts, bi)) != hipSuccess) return hip_fail(e, "hipMalloc(instances)");
    if ((e = hipMalloc((void**)&s->d_shade, bs)) != hipSuccess) {
      free_device(s);
      return hip_fail(e, "hipMalloc(materials)");
    }
    s->consts.shade = s->d_shade;
    if ((e = hipMalloc((void**)&s->d_nodes, bn)) != hipSuccess) {
      free_device(s);
      return hip_fail(e, "hipMalloc(nodes)");
    }
    const size_t bn4 = s->dnodes4.size() * sizeof(Node4Dev);
    if (bn4) {
      if ((e = hipMalloc((void**)&s->d_nodes4, bn4)) != hipSuccess) {
        free_device(s);
        return hip_fail(e, "hipMalloc(nodes4)");
      }
      if ((e = hipMemcpy(s->d_nodes4, s->dnodes4.data(), bn4, hipMemcpyHostToDevice)) != hipSuccess) {
        free_device(s);
        return hip_fail(e, "hipMemcpy(nodes4)");
      }
    }
    s->consts.nodes4 = s->d_nodes4;
    if ((e = hipMalloc((void**)&s->d_consts, sizeof(SceneConstsDev))) != hipSuccess) {
      free_device(s);
      return hip_fail(e, "hipMalloc(consts)");
    }
    if ((e = hipMemcpy(s->d_insts, leaf.data(), bi, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s->d_nodes, s->dnodes.data(), bn, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s->d_shade, leaf_shade.data(), bs, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(s->d_consts, &s->consts, sizeof(SceneConstsDev), hipMemcpyHostToDevice)) !=
            hipSuccess) {
      free_device(s);
      return hip_fail(e, "hipMemcpy(scene)");
    }
    if (!s->last_use) {
      if ((e = hipEventCreateWithFlags(&s->last_use, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "hipEventCreate");
    }
    s->device = dev;
    s->device_bytes = bi + bn + bn4 + bs + sizeof(SceneConstsDev);
    s->uploaded = true;
    return ok();
  } catch (const std::bad_alloc&) {
    return set_error(PR_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return set_error(PR_ERR_DEVICE, "unexpected exception");
  }
}

pr_status pr_scene_bvh_export(const pr_scene* s, pr_bvh_node* nodes, uint32_t node_cap,
                              uint32_t* order, uint32_t order_cap, uint32_t* n_nodes,
                              uint32_t* n_order) {
  if (!s) return set_error(PR_ERR_INVALID_ARG, "scene is NULL");
  if (!s->built) return set_error(PR_ERR_NOT_BUILT, "scene has no BVH");
  if (n_nodes) *n_nodes = (uint32_t)s->nodes.size();
  if (n_order) *n_order = (uint32_t)s->order.size();
  if (nodes) {
    if (node_cap < s->nodes.size()) return set_error(PR_ERR_INVALID_ARG, "node_cap too small");
    std::memcpy(nodes, s->nodes.data(), s->nodes.size() * sizeof(HostNode));
  }
  if (order) {
    if (order_cap < s->order.size()) return set_error(PR_ERR_INVALID_ARG, "order_cap too small");
    std::memcpy(order, s->order.data(), s->order.size() * sizeof(uint32_t));
  }
  return ok();
}

pr_status pr_scene_device_bytes(const pr_scene* s, uint64_t* bytes) {
  if (!s || !bytes) return set_error(PR_ERR_INVALID_ARG, "NULL argument");
  *bytes = s->device_bytes;
  return ok();
}

pr_status pr_scene_destroy(pr_scene* s) {
  if (!s) return set_error(PR_ERR_INVALID_ARG, "scene is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (scene_busy(s)) return set_error(PR_ERR_BUSY, "renders of this scene are in flight");
    free_device(s);
    if (s->last_use) (void)hipEventDestroy(s->last_use);
    s->last_use = nullptr;
  }
  delete s;
  return ok();
}

}  // extern "C"

extern "C" pr_status pr_scene_add_mesh(pr_scene* s, const float* vertices, uint32_t n_vertices,
                                       const uint32_t* indices, uint32_t n_triangles,
                                       const pr_instance* instances, uint32_t n_instances) {
  try {
    if (!s || !vertices || !indices || !instances) return set_error(PR_ERR_INVALID_ARG, "NULL argument");
    if (n_vertices < 3 || n_triangles == 0 || n_instances == 0)
      return set_error(PR_ERR_INVALID_ARG, "need >= 3 vertices, >= 1 triangle and >= 1 instance");
    const uint64_t total = (uint64_t)s->host_insts.size() + (uint64_t)n_triangles * n_instances;
    if (total > kMaxInstances)
      return set_error(PR_ERR_INVALID_ARG, "scene would hold %llu items, at most %u",
                       (unsigned long long)total, kMaxInstances);
    if (!finite3(vertices, (int)std::min<uint64_t>(3ull * n_vertices, 0x7fffffff)))
      return set_error(PR_ERR_INVALID_ARG, "non-finite mesh vertex");
    for (uint64_t k = 0; k < 3ull * n_triangles; ++k)
      if (indices[k] >= n_vertices) return set_error(PR_ERR_INVALID_ARG, "mesh index %u out of range", indices[k]);
    for (uint32_t i = 0; i < n_instances; ++i) {
      if (instances[i].material >= s->mats.size())
        return set_error(PR_ERR_INVALID_ARG, "mesh instance %u: material index out of range", i);
      if (!finite3(instances[i].xform, 12))
        return set_error(PR_ERR_INVALID_ARG, "mesh instance %u: non-finite transform", i);
      double A[9], Ai[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) A[3 * r + c] = instances[i].xform[4 * r + c];
      if (!(std::fabs(inv3(A, Ai)) > 1e-12))
        return set_error(PR_ERR_INVALID_ARG, "mesh instance %u: |det A| <= 1e-12", i);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (scene_busy(s)) return set_error(PR_ERR_BUSY, "renders of this scene are in flight");
    std::vector<InstDev> add;
    std::vector<float> add_shade, add_box;
    add.reserve((size_t)n_triangles * n_instances);
    for (uint32_t i = 0; i < n_instances; ++i) {
      const float* X = instances[i].xform;
      auto world = [&](uint32_t v, double out[3]) {
        const float* p = vertices + 3 * (size_t)v;
        for (int r = 0; r < 3; ++r)
          out[r] = (double)X[4 * r] * p[0] + (double)X[4 * r + 1] * p[1] + (double)X[4 * r + 2] * p[2] + X[4 * r + 3];
      };
      for (uint32_t f = 0; f < n_triangles; ++f) {
        double v0[3], v1[3], v2[3];
        world(indices[3 * (size_t)f], v0);
        world(indices[3 * (size_t)f + 1], v1);
        world(indices[3 * (size_t)f + 2], v2);
        double e1[3], e2[3];
        for (int r = 0; r < 3; ++r) {
          e1[r] = v1[r] - v0[r];
          e2[r] = v2[r] - v0[r];
        }
        const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        const double area2 = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        const double scale = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]) *
                             std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
        if (!(area2 > 1e-9 * scale) || !(area2 > 0))
          return set_error(PR_ERR_INVALID_ARG, "mesh instance %u, triangle %u: degenerate", i, f);
        InstDev d;
        std::memset(&d, 0, sizeof d);
        for (int r = 0; r < 3; ++r) {
          d.Ainv[r] = (float)v0[r];
          d.Ainv[3 + r] = (float)e1[r];
          d.Ainv[6 + r] = (float)e2[r];
          d.b[r] = (float)(n[r] / area2);
          d.lo[r] = (float)std::min({v0[r], v1[r], v2[r]});
          d.hi[r] = (float)std::max({v0[r], v1[r], v2[r]});
        }
        d.sigma = 1.f;
        d.type = kTriangle;
        const uint32_t uid = (uint32_t)(s->host_insts.size() + add.size());
        std::memcpy(&d.prm[7], &uid, 4);
        add.push_back(d);
        const pr_material& m = s->mats[instances[i].material];
        add_shade.insert(add_shade.end(), {m.albedo[0], m.albedo[1], m.albedo[2], m.reflectivity});
        add_box.insert(add_box.end(), {d.lo[0], d.lo[1], d.lo[2], d.hi[0], d.hi[1], d.hi[2]});
      }
    }
    free_device(s);
    s->built = false;
    s->host_insts.insert(s->host_insts.end(), add.begin(), add.end());
    s->host_shade.insert(s->host_shade.end(), add_shade.begin(), add_shade.end());
    s->world_aabb.insert(s->world_aabb.end(), add_box.begin(), add_box.end());
    s->consts.n_inst = (uint32_t)s->host_insts.size();
    s->n_types_present |= 1u << kTriangle;
    return ok();
  } catch (const std::bad_alloc&) {
    return set_error(PR_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return set_error(PR_ERR_DEVICE, "unexpected exception");
  }
}
