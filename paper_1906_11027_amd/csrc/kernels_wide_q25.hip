// kernels_wide_q25.hip -- instantiations of the any-lattice 2D step (wide2d.h)
// for D2Q25 (Sec. 3, Table 1), Guo forcing or the exact difference method.
#include "wide2d.h"

namespace sclbm {

template <typename T>
static hipError_t run(const StepArgs<T>& a, int order, bool edm, int variant, hipStream_t s)
{
    return a.solid ? launch_wide_lattice<T, D2Q25, true>(a, order, edm, variant, s)
                   : launch_wide_lattice<T, D2Q25, false>(a, order, edm, variant, s);
}

hipError_t launch_wide_q25(const StepArgs<float>& a, int order, bool edm, int variant, hipStream_t s)
{
    return run<float>(a, order, edm, variant, s);
}
hipError_t launch_wide_q25(const StepArgs<double>& a, int order, bool edm, int variant, hipStream_t s)
{
    return run<double>(a, order, edm, variant, s);
}

}  // namespace sclbm
