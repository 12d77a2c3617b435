// Host check of the four-wide BVH that the dense-scene kernel build
// traverses: for seeded random scenes (1 to 16384 instances, leaf sizes 1
// and 4, and tiny instances far from the origin, where float32 resolution
// is coarsest) and rays, every instance whose exact world AABB a ray hits
// robustly must be reached by a float32 emulation of the kernel's four-wide
// slab tests (all hit children visited).  Exit status 1 on a missed hit or
// a scene without a four-wide tree.
#include "host_common.h"
#include <cmath>
#include <cstdio>
#include <random>
#include <set>
using namespace pr;

static bool slab_exact(const float* lo, const float* hi, const double* o, const double* d, double& tn) {
  double t0 = 0, t1 = 1e30;
  for (int a = 0; a < 3; ++a) {
    if (std::fabs(d[a]) < 1e-12) { if (o[a] < lo[a] || o[a] > hi[a]) return false; continue; }
    double u = (lo[a] - o[a]) / d[a], v = (hi[a] - o[a]) / d[a];
    if (u > v) std::swap(u, v);
    t0 = std::max(t0, u); t1 = std::min(t1, v);
  }
  tn = t0;
  return t0 <= t1 * (1 - 1e-6) - 1e-6;   // robustly hit (not a grazing touch)
}

int main() {
  std::mt19937 rng(7);
  std::uniform_real_distribution<float> U(-1.f, 1.f);
  int bad = 0, scenes = 0, used = 0;
  for (int n : {1, 2, 3, 4, 5, 7, 16, 100, 1024, 4096, 16384}) {
    for (int rep = 0; rep < (n > 4000 ? 1 : 3); ++rep) {
      pr_geometry g{};
      g.type = PR_SPHERE;
      for (int a = 0; a < 3; ++a) { g.aabb.lo[a] = -1.f; g.aabb.hi[a] = 1.f; }
      g.params[0] = 1.f;
      std::vector<pr_instance> in(n);
      const float span = n < 10 ? 3.f : 20.f;
      for (int i = 0; i < n; ++i) {
        float s = 0.5f + 1.5f * (U(rng) * 0.5f + 0.5f);
        float xf[12] = {s, 0, 0, span * U(rng), 0, s, 0, span * U(rng), 0, 0, s, span * U(rng)};
        if (rep == 2) { xf[3] = 1000.f + U(rng) * 0.01f; xf[0] = xf[5] = xf[10] = 1e-3f; }   // tiny, far from the origin
        in[i].geometry = 0; in[i].material = 0;
        for (int k = 0; k < 12; ++k) in[i].xform[k] = xf[k];
      }
      pr_material m{{0.5f, 0.5f, 0.5f}, 0.f};
      pr_scene_consts c{{2, 4, -3}, {1, 1, 1}, 0.1f, {0, 0, 0}};
      pr_scene* s = nullptr;
      if (pr_scene_create(&g, 1, in.data(), n, &m, 1, &c, &s) != PR_OK) { printf("create failed %s\n", pr_last_error()); return 1; }
      pr_bvh_opts bo{32, (uint32_t)(rep == 1 ? 4 : 1), 1.f, 4.f, PR_BVH_HOST_ONLY};
      if (pr_bvh_build(s, &bo) != PR_OK) { printf("build failed %s\n", pr_last_error()); return 1; }
      ++scenes;
      const auto& d4 = s->dnodes4;
      if (d4.empty()) { printf("n=%d rep=%d: no four-wide tree\n", n, rep); ++bad; pr_scene_destroy(s); continue; }
      ++used;
      const auto& wa = s->world_aabb;   // user order, 6 per instance
      const auto& order = s->order;     // slot -> user index
      int misses = 0;
      for (int r = 0; r < 2000; ++r) {
        float o[3], d[3];
        for (int a = 0; a < 3; ++a) { o[a] = (rep == 2 ? 1000.f * (a == 0) : 0.f) + (span + 5) * U(rng); d[a] = U(rng); }
        float dl = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int a = 0; a < 3; ++a) d[a] /= dl;
        if (rep == 2) { for (int a = 0; a < 3; ++a) { float tgt = (a == 0 ? 1000.f : 0.f) + 0.02f * U(rng); d[a] = tgt - o[a]; } dl = std::sqrt(d[0]*d[0]+d[1]*d[1]+d[2]*d[2]); for (int a=0;a<3;++a) d[a]/=dl; }
        // kernel emulation (float32, same formulas)
        float ix = 1.0f / (d[0] != 0.f ? d[0] : std::copysign(1e-30f, d[0]));
        float iy = 1.0f / (d[1] != 0.f ? d[1] : std::copysign(1e-30f, d[1]));
        float iz = 1.0f / (d[2] != 0.f ? d[2] : std::copysign(1e-30f, d[2]));
        float oxi = -o[0] * ix, oyi = -o[1] * iy, ozi = -o[2] * iz;
        std::set<uint32_t> reached;
        std::vector<uint32_t> stack{0};
        int maxsp = 1;
        while (!stack.empty()) {
          uint32_t e = stack.back(); stack.pop_back();
          const Node4Dev& nd = d4[e];
          float sx = nd.step[0] * ix, sy = nd.step[1] * iy, sz = nd.step[2] * iz;
          float bx = std::fmaf(nd.org[0], ix, oxi), by = std::fmaf(nd.org[1], iy, oyi), bz = std::fmaf(nd.org[2], iz, ozi);
          uint32_t refs[4] = {nd.ref0, nd.ref1, nd.ref2, nd.ref3};
          for (int k = 0; k < 4; ++k) {
            if (refs[k] == kNoRef) continue;
            const uint8_t* q = nd.q + 6 * k;
            float tx0 = std::fmaf((float)q[0], sx, bx), tx1 = std::fmaf((float)q[3], sx, bx);
            float ty0 = std::fmaf((float)q[1], sy, by), ty1 = std::fmaf((float)q[4], sy, by);
            float tz0 = std::fmaf((float)q[2], sz, bz), tz1 = std::fmaf((float)q[5], sz, bz);
            float tn = std::fmax(std::fmax(std::fmin(tx0, tx1), std::fmin(ty0, ty1)), std::fmax(std::fmin(tz0, tz1), 0.f));
            float tf = std::fmin(std::fmin(std::fmax(tx0, tx1), std::fmax(ty0, ty1)), std::fmin(std::fmax(tz0, tz1), 1e30f));
            if (!(tn <= tf)) continue;
            if (refs[k] >> 31) {
              uint32_t f = refs[k] & 0xffffff, cnt = ((refs[k] >> 24) & 0x7f) + 1;
              for (uint32_t j = f; j < f + cnt; ++j) reached.insert(j);
            } else {
              stack.push_back(refs[k]);
            }
          }
          maxsp = std::max<int>(maxsp, (int)stack.size());
        }
        double od[3] = {o[0], o[1], o[2]}, dd[3] = {d[0], d[1], d[2]};
        for (uint32_t slot = 0; slot < order.size(); ++slot) {
          const float* b = &wa[6 * order[slot]];
          double tn;
          if (slab_exact(b, b + 3, od, dd, tn) && !reached.count(slot)) ++misses;
        }
      }
      printf("n=%5d rep=%d: nodes2=%zu nodes4=%zu misses=%d\n", n, rep, s->dnodes.size(), d4.size(), misses);
      bad += misses;
      pr_scene_destroy(s);
    }
  }
  printf("scenes %d, with four-wide trees %d, missed hits %d\n", scenes, used, bad);
  return bad ? 1 : 0;
}
