// Batched solve of many independent isotropic 2D problems.
// First version: problems are solved one after another on their own contexts.
#include "ctx.h"

namespace rte {

int solve_batched_impl(int count, rte_ctx* const* ctxs, const double* const* f, const double* tol, int max_iter,
                       void* const* u, rte_solve_info* infos) {
    if (count < 0 || (count > 0 && (!ctxs || !f || !tol || !u))) return set_error(RTE_EINVAL, "bad batched arguments");
    int worst = RTE_OK;
    for (int i = 0; i < count; ++i) {
        if (!ctxs[i] || ctxs[i]->dim != 2 || ctxs[i]->L != 0)
            return set_error(RTE_EINVAL, "problem %d: batched solves take 2D isotropic contexts", i);
    }
    for (int i = 0; i < count; ++i) {
        int rc = rte_solve(ctxs[i], f[i], tol[i], max_iter, u[i], infos ? &infos[i] : nullptr);
        if (rc < 0) return rc;
        if (rc > worst) worst = rc;
    }
    return worst;
}

}  // namespace rte
