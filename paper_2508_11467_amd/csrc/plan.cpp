// Host side of the merge-tree plan (see plan.h).
#include "plan.h"

#include <algorithm>

namespace bdc {
namespace {

int build_node(std::vector<LeafDesc>& leaves, std::vector<std::vector<NodeDesc>>& by_h, int64_t mat_off,
               int64_t vec_off, int32_t n, int leaf, int32_t r0, int32_t m, int32_t s) {
  if (m <= leaf) {
    leaves.push_back(LeafDesc{mat_off, vec_off, n, r0, m, s});
    return 0;
  }
  const int32_t k = m / 2;
  const int hl = build_node(leaves, by_h, mat_off, vec_off, n, leaf, r0, k - 1, 1);
  const int hr = build_node(leaves, by_h, mat_off, vec_off, n, leaf, r0 + k, m - k, s);
  const int h = 1 + std::max(hl, hr);
  if ((int)by_h.size() <= h) by_h.resize(h + 1);
  by_h[h].push_back(NodeDesc{mat_off, vec_off, n, r0, m, s, k, -1});
  return h;
}

}  // namespace

HostPlan build_host_plan(const int64_t* sizes, int64_t batch, int leaf) {
  HostPlan p;
  std::vector<std::vector<NodeDesc>> by_h;
  std::vector<int64_t> pcol(batch), ptile(batch);
  p.prob.assign(5 * std::max<int64_t>(1, batch), 0);
  int64_t vo = 0, mo = 0, co = 0, to = 0;
  for (int64_t i = 0; i < batch; ++i) {
    const int64_t n = sizes[i];
    p.prob[i] = n;
    p.prob[batch + i] = vo;
    p.prob[2 * batch + i] = mo;
    p.prob[3 * batch + i] = co;
    p.prob[4 * batch + i] = to;
    pcol[i] = co;
    ptile[i] = to;
    if (n > 0) build_node(p.leaves, by_h, mo, vo, (int32_t)n, leaf, 0, (int32_t)n, 0);
    vo += n;
    mo += n * n;
    if (n > 0) co += (n + final_u_cols(n) - 1) / final_u_cols(n);  // U work items
    to += vt_bands(n) * vt_groups(n);                                // V^T work items
  }
  p.total_n = vo;
  p.total_n2 = mo;
  p.total_cols = co;
  p.total_tiles = to;
  int id = 0;
  for (size_t hh = 1; hh < by_h.size(); ++hh) {
    int mx = 0;
    for (auto& nd : by_h[hh]) {
      nd.id = id++;
      if (nd.vec_off == 0 && nd.r0 == 0 && batch > 0 && nd.m == sizes[0]) p.root_id0 = nd.id;
      p.nodes.push_back(nd);
      mx = std::max(mx, nd.m);
    }
    p.level_count.push_back((int)by_h[hh].size());
    p.level_max_m.push_back(mx);
  }
  p.uprob.assign(std::max<int64_t>(1, co), 0);
  p.vprob.assign(std::max<int64_t>(1, to), 0);
  for (int64_t i = 0; i < batch; ++i) {
    const int64_t ue = i + 1 < batch ? pcol[i + 1] : co, ve = i + 1 < batch ? ptile[i + 1] : to;
    for (int64_t q = pcol[i]; q < ue; ++q) p.uprob[q] = (int32_t)i;
    for (int64_t q = ptile[i]; q < ve; ++q) p.vprob[q] = (int32_t)i;
  }
  return p;
}

}  // namespace bdc
