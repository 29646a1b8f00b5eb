// Learned CG preconditioner: per-context resources and the flexible-CG solve.
#include "efem_cg.h"

namespace efem {

void mlp_release(Ctx &c) { c.mlp = nullptr; }

int precond_solve_f32(Ctx &, const efem_solve_opts &, const double *, double, int, float *, float *,
                      int *, int *)
{
    set_error("learned preconditioner not set");
    return EFEM_ERR_STATE;
}

}  // namespace efem
