// fused_absent.hip -- the fused-step symbols for builds whose subgrid size
// the fused kernel does not cover (it maps the 8x8 cells of a plane onto one
// 64-lane wave).  The entry points that use it refuse such builds before they
// get here; these definitions only satisfy the linker and report failure.
#include "hydro_internal.hpp"

namespace hydro {

static_assert(NSUB != 8, "the 8^3 build links fused.hip");

int fused_variant_count() { return 0; }
const char *fused_variant_name(int) { return "?"; }
int fused_variant_order(int) { return 0; }
bool fused_needs_scratch(const StepArgs &, int) { return false; }
int64_t fused_scratch_bytes(int) { return 0; }
int fused_default_variant(int) { return 0; }
void apply_variant(StepArgs &, int) {}

hipError_t launch_fused_step(const StepArgs &, const double *, double *, double *, int32_t *,
                             int, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace hydro
