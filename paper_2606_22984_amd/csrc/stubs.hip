// Entry points whose kernels are not yet built; each reports EUNSUPPORTED.
#include "fvan_model.h"
using namespace fvan;
extern "C" {
int fvan_log_prob(fvan_model*, int32_t, const int8_t*, float*, void*) { return fail(FVAN_EUNSUPPORTED, "log_prob not built"); }
int fvan_log_prob_backward(fvan_model*, int32_t, const int8_t*, const float*, void*) { return fail(FVAN_EUNSUPPORTED, "backward not built"); }
int fvan_train_step(fvan_model*, const fvan_couplings*, double, int32_t, uint64_t, uint64_t, const fvan_adam*, double*, void*) { return fail(FVAN_EUNSUPPORTED, "train_step not built"); }
int fvan_group_create(const fvan_group_unit*, int32_t, int32_t, fvan_group**) { return fail(FVAN_EUNSUPPORTED, "group not built"); }
int fvan_group_destroy(fvan_group*) { return fail(FVAN_EUNSUPPORTED, "group not built"); }
int fvan_group_run(fvan_group*, void*) { return fail(FVAN_EUNSUPPORTED, "group not built"); }
int fvan_group_run_graph(fvan_group*, void*) { return fail(FVAN_EUNSUPPORTED, "group not built"); }
}
