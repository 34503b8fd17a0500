// design_mix_trim.hip -- greedy-design kernel variants with an FP32 tile, TRIM=true
// (one translation unit per pair so that the variants compile in parallel).
#include "design_kernel.h"

namespace lagp {

int design_launch_mix_trim(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err)
{
    return launch_variant<1, true>(a, plan, stream, err);
}

}  // namespace lagp
