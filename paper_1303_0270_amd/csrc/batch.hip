// Batched matvec over many compressed matrices (placeholder until the
// persistent kernel lands).
#include "ccm_internal.hpp"

extern "C" {
struct ccm_batch {
  int dummy;
};
int ccm_batch_create(const ccm_desc *, int32_t, int32_t, const char *, ccm_batch **) {
  return CCM_E_UNSUPPORTED;
}
int ccm_batch_set_io(ccm_batch *, const void *const *, int64_t *const *, void *) {
  return CCM_E_UNSUPPORTED;
}
int ccm_batch_matvec(ccm_batch *, int32_t, void *) { return CCM_E_UNSUPPORTED; }
int ccm_batch_info(const ccm_batch *, int64_t *, uint64_t *, int32_t *) {
  return CCM_E_UNSUPPORTED;
}
int ccm_batch_destroy(ccm_batch *) { return CCM_E_UNSUPPORTED; }
}
