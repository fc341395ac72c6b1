// Serving runtime: placeholder entry points until the packed server lands.
#include "te.h"
#include "te_job.h"

using namespace te;

extern "C" {
te_status te_server_create(const te_server_config *, te_server *) {
  return set_error(TE_EINVAL, "serving is not available in this build");
}
te_status te_submit(te_server, const te_problem *, te_precision, uint64_t *) {
  return set_error(TE_EINVAL, "serving is not available in this build");
}
te_status te_poll(te_server, uint64_t, double *, te_stats *) {
  return set_error(TE_EINVAL, "serving is not available in this build");
}
te_status te_wait(te_server, uint64_t, double *, te_stats *) {
  return set_error(TE_EINVAL, "serving is not available in this build");
}
te_status te_server_destroy(te_server) {
  return set_error(TE_EINVAL, "serving is not available in this build");
}
}
