// Learned right preconditioner (3x3 convolution network).  The network kernels are added in a
// separate step; until then attaching a network reports RTE_EUNSUPPORTED.
#include "nn.h"

namespace rte {
int pc_apply(rte_ctx* c, const double* v, double* z) {
    (void)c; (void)v; (void)z;
    return set_error(RTE_EUNSUPPORTED, "learned preconditioner not available");
}
void pc_free(rte_ctx* c) { c->pc_attached = false; }
}  // namespace rte

extern "C" int rte_pc_attach(rte_ctx* ctx, const float* weights_dev, int hidden, int layers) {
    (void)ctx; (void)weights_dev; (void)hidden; (void)layers;
    return rte::set_error(RTE_EUNSUPPORTED, "learned preconditioner not available");
}
