// kernels_wide_q9.hip -- instantiations of the any-lattice 2D step (wide2d.h)
// for D2Q9 with the exact difference method, and for D2Q9 with walls.
#include "wide2d.h"

namespace sclbm {

template <typename T>
static hipError_t run(const StepArgs<T>& a, int order, bool edm, int variant, hipStream_t s)
{
    // D2Q9 with Guo forcing and no walls runs in the D2Q9 family (kernels_2d.hip)
    if (a.solid) return launch_wide_lattice<T, D2Q9, true>(a, order, edm, variant, s);
    if (!edm) return hipErrorInvalidValue;
    return launch_wide_order<T, D2Q9, true, false>(a, order, variant, s);
}

hipError_t launch_wide_q9(const StepArgs<float>& a, int order, bool edm, int variant, hipStream_t s)
{
    return run<float>(a, order, edm, variant, s);
}
hipError_t launch_wide_q9(const StepArgs<double>& a, int order, bool edm, int variant, hipStream_t s)
{
    return run<double>(a, order, edm, variant, s);
}

}  // namespace sclbm
