// Batched CG solves (persistent workgroups).  Placeholder until the batched
// kernel lands: reports DSM_E_UNSUPPORTED.
#include "core.hpp"

using namespace dsm;

DSM_API dsm_status dsm_cg_solve_batched(int32_t count, const dsm_matrix *mats, const double *const *b,
                                        double *const *x, const dsm_cg_opts *opts, dsm_cg_result *results,
                                        void *stream) {
    return guard([&] { fail(DSM_E_UNSUPPORTED, "batched solves are not built yet"); });
}
