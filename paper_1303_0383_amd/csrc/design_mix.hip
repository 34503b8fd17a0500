// design_mix.hip -- greedy-design kernel variants with an FP32 tile, TRIM=false
// (one translation unit per pair so that the variants compile in parallel).
#include "design_kernel.h"

namespace lagp {

int design_launch_mix(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err)
{
    return launch_variant<1, false>(a, plan, stream, err);
}

}  // namespace lagp
