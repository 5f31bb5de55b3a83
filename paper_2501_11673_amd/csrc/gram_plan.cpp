// Work split of the Kaczmarz++ Gram kernels (host code): every lower 16 x 16
// tile of a block over column chunks of whole LDS panels, enough chunks for
// about kGramTargetGroups workgroups per launch, each chunk at least
// kGramMinPanels panels long (shorter chunks write more partial tiles than
// they read of A).
#include <algorithm>
#include <cstddef>
#include <cstdint>

#include "kernels.hpp"

namespace kpp {

namespace {
void split(int32_t s, int64_t n, int64_t want, int32_t* nchunks, int64_t* chunk, int32_t* ntiles) {
  const int32_t g = gram_groups(s);
  const int32_t kc = gram_panel(g);
  *ntiles = g * (g + 1) / 2;
  const int64_t panels = std::max<int64_t>(1, (n + kc - 1) / kc);
  const int64_t cmax = std::max<int64_t>(1, panels / kGramMinPanels);
  const int64_t c = std::max<int64_t>(1, std::min(want, cmax));
  const int64_t per = ((panels + c - 1) / c) * kc;   // whole panels per chunk
  *chunk = per;
  *nchunks = static_cast<int32_t>(std::max<int64_t>(1, (n + per - 1) / per));
}
}  // namespace

void gram_syrk_plan(int32_t s, int64_t n, int32_t nb, int32_t* nchunks, int64_t* chunk, int32_t* ntiles) {
  split(s, n, kGramTargetGroups / std::max(nb, 1), nchunks, chunk, ntiles);
}

void gram_syrk_plan_capped(int32_t s, int64_t n, int32_t nb, size_t max_work, int32_t* nchunks, int64_t* chunk,
                           int32_t* ntiles) {
  gram_syrk_plan(s, n, nb, nchunks, chunk, ntiles);
  const size_t per_chunk = static_cast<size_t>(std::max(nb, 1)) * *ntiles * kGramTile * kGramTile;
  if (static_cast<size_t>(*nchunks) * per_chunk <= max_work) return;
  split(s, n, std::max<int64_t>(1, static_cast<int64_t>(max_work / per_chunk)), nchunks, chunk, ntiles);
}

size_t gram_syrk_work(int32_t s, int64_t n, int32_t nb) {
  int32_t nc, nt;
  int64_t chunk;
  gram_syrk_plan(s, n, nb, &nc, &chunk, &nt);
  return static_cast<size_t>(nb) * nt * nc * kGramTile * kGramTile;
}

}  // namespace kpp
