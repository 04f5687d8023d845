// Langevin MD step (placeholder until the integrator lands).
#include "ffbh_internal.h"

namespace ffbh {

hipError_t launch_md(Handle &, const md_state *, const md_params *, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace ffbh
