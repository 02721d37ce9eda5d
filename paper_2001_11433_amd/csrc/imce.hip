// Incremental maintenance (Section 5): placeholder entry points.
#include "internal.h"

using namespace mce;

struct imce_state { int unused; };

extern "C" {
int imce_create(const mce_csr*, const mce_opts*, imce_state**, mce_result*) {
  set_error("imce_create: not built yet");
  return MCE_ENOTSUP;
}
int imce_add_edges(imce_state*, const uint32_t*, const uint32_t*, uint64_t, int, imce_result*, mce_clique_buf*,
                   mce_clique_buf*) {
  set_error("imce_add_edges: not built yet");
  return MCE_ENOTSUP;
}
int imce_info(const imce_state*, uint64_t*, uint64_t*, uint64_t*, uint64_t*) { return MCE_ENOTSUP; }
void imce_destroy(imce_state*) {}
}
