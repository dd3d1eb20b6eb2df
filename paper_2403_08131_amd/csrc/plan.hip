// Interdependence analysis that decides the set of tuning searches (the
// paper's Sec. IV-B to IV-D): sensitivities of every routine to every
// parameter from a one-at-a-time sweep, influence scores, the cut-off, the
// merge of routines linked by influential external parameters into joint
// searches, and the cap on the dimensions of a search.  Host code: the
// arithmetic is a few thousand divisions; the routine outputs come from the
// application (or a synthetic objective) evaluated on the sweep.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "gpbo_internal.h"

namespace gpbo {

namespace {

// Disjoint sets over the routines, with path halving; the representative of
// a set is its smallest routine.
struct Dsu {
  std::vector<int> parent;
  explicit Dsu(int n) : parent(n) { std::iota(parent.begin(), parent.end(), 0); }
  int find(int a) {
    while (parent[a] != a) {
      parent[a] = parent[parent[a]];
      a = parent[a];
    }
    return a;
  }
  void join(int a, int b) {
    a = find(a);
    b = find(b);
    if (a == b) return;
    if (a < b) std::swap(a, b);
    parent[a] = b;
  }
};

}  // namespace

}  // namespace gpbo

using namespace gpbo;

extern "C" {

gpbo_status gpbo_sensitivity(int32_t P, int32_t R, int32_t V, const double* base,
                             const double* out, double* S) {
  if (P <= 0 || R <= 0 || V <= 0 || !base || !out || !S) return GPBO_E_INVALID_ARG;
  for (int r = 0; r < R; ++r)
    if (!(base[r] != 0.0) || !std::isfinite(base[r])) return GPBO_E_INVALID_ARG;
  for (int r = 0; r < R; ++r) {
    const double b = base[r];
    for (int j = 0; j < P; ++j) {
      // mean relative change of routine r's output over the V variations of
      // parameter j
      const double* o = out + (size_t)j * V * R + r;
      double acc = 0.0;
      for (int i = 0; i < V; ++i) acc += std::fabs((b - o[(size_t)i * R]) / b);
      S[(size_t)r * P + j] = acc / V;
    }
  }
  return GPBO_OK;
}

gpbo_status gpbo_plan_searches(int32_t P, int32_t R, const double* S, const int32_t* owner,
                               double cutoff, int32_t max_dims, int32_t* routine_search,
                               int32_t* param_search, int32_t* n_searches) {
  if (P <= 0 || R <= 0 || !S || !owner || !routine_search || !param_search || !n_searches ||
      max_dims <= 0 || !(cutoff >= 0.0))
    return GPBO_E_INVALID_ARG;
  for (int j = 0; j < P; ++j)
    if (owner[j] < 0 || owner[j] >= R) return GPBO_E_INVALID_ARG;
  // influence: sensitivity relative to the routine's most sensitive own parameter
  std::vector<double> top(R, 0.0);
  for (int j = 0; j < P; ++j) {
    const int o = owner[j];
    top[o] = std::max(top[o], S[(size_t)o * P + j]);
  }
  auto infl = [&](int r, int j) {
    return top[r] > 0.0 ? S[(size_t)r * P + j] / top[r] : 0.0;
  };
  // routines joined through external edges that survive the cut-off
  Dsu dsu(R);
  for (int j = 0; j < P; ++j)
    for (int r = 0; r < R; ++r)
      if (r != owner[j] && infl(r, j) >= cutoff) dsu.join(owner[j], r);
  // searches numbered in order of their smallest routine
  std::vector<int> id(R, -1);
  int n = 0;
  for (int r = 0; r < R; ++r) {
    const int root = dsu.find(r);
    if (id[root] < 0) id[root] = n++;
    routine_search[r] = id[root];
  }
  for (int j = 0; j < P; ++j) param_search[j] = routine_search[owner[j]];
  // cap: keep the max_dims parameters with the largest influence on any
  // routine of their search (ties to the lower index), fix the rest
  for (int s = 0; s < n; ++s) {
    std::vector<int> members;
    for (int j = 0; j < P; ++j)
      if (param_search[j] == s) members.push_back(j);
    if ((int)members.size() <= max_dims) continue;
    std::vector<std::pair<double, int>> score;
    for (int j : members) {
      double best = 0.0;
      for (int r = 0; r < R; ++r)
        if (routine_search[r] == s) best = std::max(best, infl(r, j));
      score.emplace_back(-best, j);
    }
    std::sort(score.begin(), score.end());
    for (size_t q = (size_t)max_dims; q < score.size(); ++q) param_search[score[q].second] = -1;
  }
  *n_searches = n;
  return GPBO_OK;
}

}  // extern "C"
