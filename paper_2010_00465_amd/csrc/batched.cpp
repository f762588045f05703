// Batched entry points (filled in by the persistent batched kernel).
#include "common.hpp"

extern "C" {

size_t sincosm_batched_workspace_size(int64_t batch, const int32_t* n_host, int dtype, int acc, int prod) {
  (void)batch; (void)n_host; (void)dtype; (void)acc; (void)prod;
  return 0;
}

sincosm_status sincosm_eval_batched(int64_t batch, int dtype, const int32_t* n_host, const int64_t* offset_host,
                                    const void* A, void* C, void* S, int acc, int prod, void* ws, size_t ws_bytes,
                                    sincosm_plan* plans_dev, void* stream) {
  (void)batch; (void)dtype; (void)n_host; (void)offset_host; (void)A; (void)C; (void)S; (void)acc; (void)prod;
  (void)ws; (void)ws_bytes; (void)plans_dev; (void)stream;
  return SINCOSM_E_UNSUPPORTED;
}

}  // extern "C"
