// Adjoint entry points (filled in by the reverse pass).
#include "common.hpp"

extern "C" {

size_t sincosm_backward_workspace_size(int64_t n, int dtype, int acc, int32_t s) {
  (void)n; (void)dtype; (void)acc; (void)s;
  return 0;
}

sincosm_status sincosm_backward(int64_t n, int dtype, const void* A, int64_t lda, const void* Gc, int64_t ldgc,
                                const void* Gs, int64_t ldgs, void* gA, int64_t ldga, int acc, void* ws,
                                size_t ws_bytes, sincosm_plan* plan_host, void* stream) {
  (void)n; (void)dtype; (void)A; (void)lda; (void)Gc; (void)ldgc; (void)Gs; (void)ldgs; (void)gA; (void)ldga;
  (void)acc; (void)ws; (void)ws_bytes; (void)plan_host; (void)stream;
  return SINCOSM_E_UNSUPPORTED;
}

}  // extern "C"
