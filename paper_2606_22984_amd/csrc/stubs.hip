// Entry points whose kernels are not yet built; each reports EUNSUPPORTED.
#include "fvan_model.h"
using namespace fvan;
extern "C" {
int fvan_group_create(const fvan_group_unit*, int32_t, int32_t, fvan_group**) { return fail(FVAN_EUNSUPPORTED, "group not built"); }
int fvan_group_destroy(fvan_group*) { return fail(FVAN_EUNSUPPORTED, "group not built"); }
int fvan_group_run(fvan_group*, void*) { return fail(FVAN_EUNSUPPORTED, "group not built"); }
int fvan_group_run_graph(fvan_group*, void*) { return fail(FVAN_EUNSUPPORTED, "group not built"); }
}
