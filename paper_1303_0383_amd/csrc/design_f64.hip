// design_f64.hip -- greedy-design kernel variants with an FP64 tile, TRIM=false
// (one translation unit per pair so that the variants compile in parallel).
#include "design_kernel.h"

namespace lagp {

int design_launch_f64(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err)
{
    return launch_variant<0, false>(a, plan, stream, err);
}

}  // namespace lagp
