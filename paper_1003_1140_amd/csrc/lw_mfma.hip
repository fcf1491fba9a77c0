// lw_mfma.hip -- matrix-core path (not yet available in this build).
#include "lw_mfma.h"

namespace lw {

struct MfmaPlanCache {};

MfmaPlanCache* mfma_cache_create() { return new MfmaPlanCache(); }
void mfma_cache_destroy(MfmaPlanCache* c) { delete c; }
void mfma_cache_invalidate(MfmaPlanCache*) {}

lw_status mfma_workspace_size(lw_ctx* c, const lw_batch*, lw_path, size_t* bytes) {
  *bytes = 0;
  c->err = "matrix-core path not available";
  return LW_EUNSUPPORTED;
}

lw_status mfma_accumulate(lw_ctx* c, const lw_batch*, lw_path, void*, size_t, float*) {
  c->err = "matrix-core path not available";
  return LW_EUNSUPPORTED;
}

}  // namespace lw
