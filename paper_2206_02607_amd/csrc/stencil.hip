// Host-side construction of the finite-element stencil of the integration
// samples (appendix, Sec. "Solid Mechanics / Reduced-order Model"): for
// every sample vertex the tetrahedra incident on it, and for every instance
// the vertices of those tetrahedra, its one-ring, at which the decoder is
// evaluated.  The result is laid out as crom_fe_mesh takes it.
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "common.hpp"

using namespace crom;

extern "C" {

crom_status crom_fe_stencil(int64_t n_vert, int64_t n_tet, const int32_t* tets, int32_t n_inst,
                            const int64_t* sample_offsets, const int32_t* sample_vert, int64_t* n_ring,
                            int64_t* max_ring, int64_t* n_inc, int64_t* ring_offsets, int32_t* ring_vert,
                            int64_t* inc_offsets, int32_t* inc_tets, int8_t* inc_corner) {
  if (n_vert < 0 || n_tet < 0 || n_inst < 0) return fail(CROM_ERR_INVALID_ARG, "negative size");
  if (n_vert > INT32_MAX) return fail(CROM_ERR_INVALID_ARG, "too many vertices");
  if (!n_ring || !max_ring || !n_inc || !sample_offsets || (n_tet > 0 && !tets))
    return fail(CROM_ERR_INVALID_ARG, "tets, sample_offsets and the size outputs are required");
  const bool fill = ring_offsets != nullptr;
  if (fill && (!ring_vert || !inc_offsets || !inc_tets || !inc_corner))
    return fail(CROM_ERR_INVALID_ARG, "the fill call needs every output array");
  for (int64_t t = 0; t < n_tet * 4; ++t)
    if (tets[t] < 0 || tets[t] >= n_vert) return fail(CROM_ERR_INVALID_ARG, "tetrahedron vertex out of range");
  if (sample_offsets[0] != 0) return fail(CROM_ERR_INVALID_ARG, "sample_offsets[0] must be 0");
  for (int32_t i = 0; i < n_inst; ++i)
    if (sample_offsets[i + 1] < sample_offsets[i]) return fail(CROM_ERR_INVALID_ARG, "sample_offsets decrease");
  const int64_t total = sample_offsets[n_inst];
  if (total > 0 && !sample_vert) return fail(CROM_ERR_INVALID_ARG, "sample_vert is NULL");
  for (int64_t p = 0; p < total; ++p)
    if (sample_vert[p] < 0 || sample_vert[p] >= n_vert) return fail(CROM_ERR_INVALID_ARG, "sample vertex out of range");

  // vertex -> incident tetrahedra (ascending), by counting sort
  std::vector<int64_t> vstart(n_vert + 1, 0);
  for (int64_t t = 0; t < n_tet * 4; ++t) ++vstart[tets[t] + 1];
  for (int64_t v = 0; v < n_vert; ++v) vstart[v + 1] += vstart[v];
  std::vector<int64_t> vtet(n_tet * 4), fillp(vstart.begin(), vstart.end() - 1);
  for (int64_t t = 0; t < n_tet; ++t)
    for (int k = 0; k < 4; ++k) {
      const int32_t v = tets[t * 4 + k];
      // a vertex listed twice in one tetrahedron is a degenerate element
      if (fillp[v] > vstart[v] && vtet[fillp[v] - 1] == t)
        return fail(CROM_ERR_INVALID_ARG, "tetrahedron with a repeated vertex");
      vtet[fillp[v]++] = t;
    }

  std::vector<int32_t> stamp(n_vert, -1), local(n_vert, 0), ring;
  int64_t nr = 0, mr = 0, ni = 0;
  if (fill) {
    ring_offsets[0] = 0;
    inc_offsets[0] = 0;
  }
  for (int32_t i = 0; i < n_inst; ++i) {
    ring.clear();
    for (int64_t p = sample_offsets[i]; p < sample_offsets[i + 1]; ++p) {
      const int32_t s = sample_vert[p];
      if (vstart[s + 1] == vstart[s]) return fail(CROM_ERR_INVALID_ARG, "sample vertex without tetrahedra");
      for (int64_t e = vstart[s]; e < vstart[s + 1]; ++e)
        for (int k = 0; k < 4; ++k) {
          const int32_t v = tets[vtet[e] * 4 + k];
          if (stamp[v] != i) {
            stamp[v] = i;
            ring.push_back(v);
          }
        }
    }
    std::sort(ring.begin(), ring.end());
    for (size_t j = 0; j < ring.size(); ++j) local[ring[j]] = (int32_t)j;
    if (fill) {
      std::copy(ring.begin(), ring.end(), ring_vert + nr);
      for (int64_t p = sample_offsets[i]; p < sample_offsets[i + 1]; ++p) {
        const int32_t s = sample_vert[p];
        int64_t e_out = inc_offsets[p];
        for (int64_t e = vstart[s]; e < vstart[s + 1]; ++e, ++e_out) {
          const int64_t t = vtet[e];
          int8_t corner = 0;
          for (int k = 0; k < 4; ++k) {
            const int32_t v = tets[t * 4 + k];
            inc_tets[e_out * 4 + k] = local[v];
            if (v == s) corner = (int8_t)k;
          }
          inc_corner[e_out] = corner;
        }
        inc_offsets[p + 1] = e_out;
      }
    }
    for (int64_t p = sample_offsets[i]; p < sample_offsets[i + 1]; ++p) ni += vstart[sample_vert[p] + 1] - vstart[sample_vert[p]];
    nr += (int64_t)ring.size();
    mr = std::max<int64_t>(mr, (int64_t)ring.size());
    if (fill) ring_offsets[i + 1] = nr;
  }
  *n_ring = nr;
  *max_ring = mr;
  *n_inc = ni;
  return CROM_OK;
}

}  // extern "C"
