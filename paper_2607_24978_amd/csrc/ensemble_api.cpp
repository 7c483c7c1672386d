// Ensemble entry points (placeholder until the batched kernel lands).
#include "internal.h"

extern "C" {
cl_status cl_ensemble_create(int, cl_lattice* const*, cl_ensemble** out) {
    if (out) *out = nullptr;
    return CL_EUNSUPPORTED;
}
cl_status cl_ensemble_set_dt(cl_ensemble*, int, double) { return CL_EUNSUPPORTED; }
cl_status cl_ensemble_step(cl_ensemble*, cl_integrator, int, cl_observables*) { return CL_EUNSUPPORTED; }
cl_status cl_ensemble_destroy(cl_ensemble*) { return CL_OK; }
}
