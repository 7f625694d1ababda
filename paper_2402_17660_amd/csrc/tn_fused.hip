// Fused path (MFMA pair tiles); filled in once the plain path is verified.
#include "tn_internal.h"

namespace tn {

size_t fused_workspace_bytes(const tn_model *, int64_t, int64_t, int64_t, const BoxInfo &, int, int) { return 0; }

int fused_run(const tn_model *, hipStream_t, const Problem &, int, void *, size_t) { return TN_E_UNSUPPORTED; }

}  // namespace tn
