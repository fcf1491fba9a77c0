// lw_mfma.h -- matrix-core path of the accumulation (spread + DFT contraction).
#pragma once
#include "lw_internal.h"

namespace lw {

MfmaPlanCache* mfma_cache_create();
void mfma_cache_destroy(MfmaPlanCache* c);
void mfma_cache_invalidate(MfmaPlanCache* c);
// Counts table rebuilds: captured work that read older tables must not run.
uint64_t mfma_epoch(const MfmaPlanCache* c);
lw_status mfma_set_options(lw_ctx* c, int bands, int products_f16, int products_bf16);
lw_status mfma_set_bands(lw_ctx* c, int bands);
lw_status mfma_set_tile(lw_ctx* c, int tile);
lw_status mfma_set_chunk_bytes(lw_ctx* c, int64_t bytes);
// Plans the batch and reports {particles per chunk, chunks, bands, workspace bytes}.
lw_status mfma_plan_info(lw_ctx* c, const lw_batch* b, lw_path path, int64_t* out);
// Plans the batch: measures its retarded-time span (synchronises), grows the tables if
// needed and remembers the batch as planned.
lw_status mfma_workspace_size(lw_ctx* c, const lw_batch* b, lw_path path, size_t* bytes);
// The same size without measuring a planned batch again (no synchronisation then).
lw_status mfma_workspace_need(lw_ctx* c, const lw_batch* b, lw_path path, size_t* bytes);
// amp: null, or a per-particle amplitude state [P][nd][nw][4] the columns' amplitudes are
// added to (then S and the summed amplitudes are left alone)
lw_status mfma_accumulate(lw_ctx* c, const lw_batch* b, lw_path path, void* ws, size_t ws_bytes,
                          float* per_particle, double* amp = nullptr);

}  // namespace lw
