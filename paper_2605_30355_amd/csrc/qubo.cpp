// qubo.cpp -- QUBO -> Ising mapping at the boundary (cosm_qubo_to_ising).
//
// minimise E(x) = sum_k Q_k x_{i_k} x_{j_k}, x in {0,1}^n.  With x = (1 + s)/2:
//   i != j:  x_i x_j = (1 + s_i + s_j + s_i s_j) / 4
//   i == j:  x_i     = (1 + s_i) / 2
// so 4 E(x) = H(s) + offset with the Ising energy of Eq. (1),
//   J_uv = -sum of Q_k over the off-diagonal terms on {u, v} (either order),
//   h_i  = -(sum of Q_k over off-diagonal terms touching i + 2 sum of Q_ii),
//   offset = sum of off-diagonal Q_k + 2 sum of diagonal Q_k.
// Pairs whose merged J is 0 are dropped.  Edges come out sorted by (u, v), u < v.
#include <algorithm>
#include <map>
#include <utility>
#include <vector>

#include "internal.hpp"

extern "C" int cosm_qubo_to_ising(int32_t n, int64_t nnz, const int32_t *qi, const int32_t *qj,
                                  const int32_t *qv, int32_t *eu_out, int32_t *ev_out,
                                  int32_t *J_out, int64_t *m_out, int32_t *h_out,
                                  int64_t *offset_out) {
  using namespace cosm;
  clear_error();
  if (n < 1) return set_error(COSM_EINVAL, "n must be >= 1");
  if (nnz < 0 || (nnz > 0 && (qi == nullptr || qj == nullptr || qv == nullptr)))
    return set_error(COSM_EINVAL, "bad QUBO term arrays");
  if (eu_out == nullptr || ev_out == nullptr || J_out == nullptr || m_out == nullptr ||
      h_out == nullptr || offset_out == nullptr)
    return set_error(COSM_EINVAL, "output pointers must not be NULL");
  std::map<std::pair<int32_t, int32_t>, int64_t> pair;
  std::vector<int64_t> h((size_t)n, 0);
  int64_t offset = 0;
  for (int64_t k = 0; k < nnz; k++) {
    const int32_t i = qi[k], j = qj[k];
    const int64_t q = qv[k];
    if (i < 0 || i >= n || j < 0 || j >= n) return set_error(COSM_EINVAL, "QUBO index out of range");
    if (i == j) {
      h[(size_t)i] -= 2 * q;
      offset += 2 * q;
    } else {
      pair[{std::min(i, j), std::max(i, j)}] -= q;
      h[(size_t)i] -= q;
      h[(size_t)j] -= q;
      offset += q;
    }
  }
  int64_t m = 0;
  for (const auto &kv : pair) {
    if (kv.second == 0) continue;
    if (kv.second > INT32_MAX || kv.second < INT32_MIN)
      return set_error(COSM_ERANGE, "a merged coupling does not fit int32");
    eu_out[m] = kv.first.first;
    ev_out[m] = kv.first.second;
    J_out[m] = (int32_t)kv.second;
    m++;
  }
  for (int32_t i = 0; i < n; i++) {
    if (h[(size_t)i] > INT32_MAX || h[(size_t)i] < INT32_MIN)
      return set_error(COSM_ERANGE, "a field does not fit int32");
    h_out[i] = (int32_t)h[(size_t)i];
  }
  *m_out = m;
  *offset_out = offset;
  return COSM_OK;
}
