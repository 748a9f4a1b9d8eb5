// Direction-dependent kernels (CohJones / AllJones): placeholder until the MFMA Gram path lands.
#include "wcal_internal.h"

size_t dd_stats_bytes(const wcal_problem&) { return 0; }
hipError_t launch_dd_solve(const wcal_plan*, const DdArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_dd_accumulate(const wcal_plan*, const DdArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_dd_residual(const wcal_plan*, const DdArgs&, hipStream_t) { return hipErrorNotSupported; }
