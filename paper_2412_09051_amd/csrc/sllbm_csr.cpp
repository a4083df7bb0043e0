// Curvilinear (CSR-by-cell) plan builder: placeholder until the isoparametric
// departure-point search is in place.
#include "sllbm_internal.h"

namespace sllbm {
int build_csr_tables(const Mesh &m, const VelSet &v, double dt, HostTables &t, int64_t *n_exc, int64_t *n_th) {
  (void)m; (void)v; (void)dt; (void)t; (void)n_exc; (void)n_th;
  return fail(SLLBM_EUNSUPPORTED, "curvilinear plans are not built yet");
}
}  // namespace sllbm
