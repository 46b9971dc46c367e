// Interpolation-based space-time FMM (Section 3, Section 4).
#include "internal.h"

namespace tdbem {

struct Fmm {};

Fmm* fmm_create(tdbem_ctx*) { throw Error(TDBEM_E_INVAL, "FMM mode is not available in this build"); }
void fmm_destroy(Fmm* f) { delete f; }
void fmm_reset(tdbem_ctx*) {}
void fmm_far(tdbem_ctx*, int, double*) {}
void fmm_advance(tdbem_ctx*, int) {}
void fmm_info(const tdbem_ctx*, tdbem_info*) {}
void fmm_near_pairs(const tdbem_ctx*, std::vector<int64_t>&, std::vector<int32_t>&) {}

}  // namespace tdbem
