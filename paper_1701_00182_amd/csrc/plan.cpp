// Host-only structure of a factorisation (see plan.h): cluster tree, level
// schedule, option validation and the structure queries of the C ABI.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

namespace acr {

namespace {
struct Box { int x0, x1, y0, y1; };
inline int box_size(const Box& b) { return (b.x1 - b.x0) * (b.y1 - b.y0); }
}  // namespace

bool Tree::build(int nx_, int ny_, int leaf_) {
  nx = nx_; ny = ny_; leaf = leaf_; M = nx * ny;
  std::vector<std::vector<Box>> levels{{Box{0, nx, 0, ny}}};
  for (;;) {
    const auto& cur = levels.back();
    int mx = 0;
    for (auto& b : cur) mx = std::max(mx, box_size(b));
    if (mx <= leaf) break;
    std::vector<Box> nxt;
    nxt.reserve(cur.size() * 2);
    for (auto& b : cur) {
      if (box_size(b) < 2) return false;
      const int w = b.x1 - b.x0, h = b.y1 - b.y0;
      if (w >= h) {
        const int xm = b.x0 + (w + 1) / 2;
        nxt.push_back({b.x0, xm, b.y0, b.y1});
        nxt.push_back({xm, b.x1, b.y0, b.y1});
      } else {
        const int ym = b.y0 + (h + 1) / 2;
        nxt.push_back({b.x0, b.x1, b.y0, ym});
        nxt.push_back({b.x0, b.x1, ym, b.y1});
      }
    }
    levels.push_back(std::move(nxt));
  }
  L = (int)levels.size() - 1;
  off.assign(L + 1, {});
  sz.assign(L + 1, {});
  for (int d = 0; d <= L; ++d) {
    int o = 0;
    for (auto& b : levels[d]) {
      off[d].push_back(o);
      sz[d].push_back(box_size(b));
      o += box_size(b);
    }
  }
  perm.clear();
  leaf_max = 0;
  for (auto& b : levels[L]) {
    leaf_max = std::max(leaf_max, box_size(b));
    for (int j = b.y0; j < b.y1; ++j)
      for (int i = b.x0; i < b.x1; ++i) perm.push_back(j * nx + i);
  }
  return true;
}

std::vector<std::vector<int>> level_schedule(int nplanes, int* last) {
  std::vector<std::vector<int>> out;
  std::vector<int> alive(std::max(nplanes, 0));
  for (int k = 0; k < (int)alive.size(); ++k) alive[k] = k;
  while (alive.size() > 1) {
    out.push_back(alive);
    std::vector<int> kept;
    for (size_t q = 1; q < alive.size(); q += 2) kept.push_back(alive[q]);
    alive = std::move(kept);
  }
  if (last) *last = alive.empty() ? -1 : alive[0];
  return out;
}

bool options_valid(const acr_options_t* o) {
  if (!o) return false;
  if (o->nx < 1 || o->ny < 1 || o->nplanes < 1 || o->leaf < 1) return false;
  if (!(o->eps >= 0.0) || !std::isfinite(o->eps)) return false;
  if (o->max_rank < 0) return false;
  if (o->precision < ACR_PREC_FP64 || o->precision > ACR_PREC_FP32_FP16) return false;
  if ((o->alloc == nullptr) != (o->release == nullptr)) return false;
  if (!(o->inner_eps_ratio >= 0.0) || !std::isfinite(o->inner_eps_ratio)) return false;
  if (o->stencil_points != 0 && o->stencil_points != 7 && o->stencil_points != 27) return false;
  if (o->gemm_tiles < 0 || o->gemm_tiles > 1) return false;
  if ((int64_t)o->nx * o->ny > (int64_t)1 << 28) return false;
  if ((int64_t)o->nx * o->ny * o->nplanes > (int64_t)1 << 34) return false;
  return true;
}

// Fills the structure record and whichever arrays are non-null (sizes in the
// record); `elim[i][q]` says whether plane sched[i][q] was eliminated.
void fill_structure(const Tree& tr, const std::vector<std::vector<int>>& sched,
                    const std::vector<std::vector<char>>& elim, int last, const int32_t* perm_src,
                    acr_structure_t* info, int32_t* perm, int32_t* node_offset, int32_t* node_size,
                    int32_t* level_size, int32_t* sched_plane, int32_t* sched_elim) {
  std::memset(info, 0, sizeof(*info));
  info->M = tr.M;
  info->depth = tr.L;
  info->nodes = (1 << (tr.L + 1)) - 1;
  info->levels = (int32_t)sched.size();
  for (auto& l : sched) info->schedule_len += (int32_t)l.size();
  info->last_plane = last;
  if (perm)
    for (int p = 0; p < tr.M; ++p) perm[p] = perm_src ? perm_src[p] : tr.perm[p];
  for (int d = 0; d <= tr.L; ++d)
    for (int s = 0; s < (1 << d); ++s) {
      const int id = (1 << d) - 1 + s;
      if (node_offset) node_offset[id] = tr.off[d][s];
      if (node_size) node_size[id] = tr.sz[d][s];
    }
  int pos = 0;
  for (size_t i = 0; i < sched.size(); ++i) {
    if (level_size) level_size[i] = (int32_t)sched[i].size();
    for (size_t q = 0; q < sched[i].size(); ++q, ++pos) {
      if (sched_plane) sched_plane[pos] = sched[i][q];
      if (sched_elim) sched_elim[pos] = elim[i][q] ? 1 : 0;
    }
  }
}

}  // namespace acr

extern "C" acr_status_t acr_plan_structure(int32_t nx, int32_t ny, int32_t nplanes, int32_t leaf,
                                           acr_structure_t* info, int32_t* perm, int32_t* node_offset,
                                           int32_t* node_size, int32_t* level_size, int32_t* sched_plane,
                                           int32_t* sched_elim) {
  if (!info || nx < 1 || ny < 1 || nplanes < 1 || leaf < 1 || (int64_t)nx * ny > (int64_t)1 << 28)
    return ACR_ERROR_INVALID_VALUE;
  try {
    acr::Tree tr;
    if (!tr.build(nx, ny, leaf)) return ACR_ERROR_INVALID_VALUE;
    int last = -1;
    const auto sched = acr::level_schedule(nplanes, &last);
    std::vector<std::vector<char>> elim(sched.size());
    for (size_t i = 0; i < sched.size(); ++i) {
      elim[i].assign(sched[i].size(), 0);
      for (size_t q = 0; q < sched[i].size(); q += 2) elim[i][q] = 1;
    }
    acr::fill_structure(tr, sched, elim, last, nullptr, info, perm, node_offset, node_size, level_size,
                        sched_plane, sched_elim);
    return ACR_SUCCESS;
  } catch (...) {
    return ACR_ERROR_OUT_OF_MEMORY;
  }
}
