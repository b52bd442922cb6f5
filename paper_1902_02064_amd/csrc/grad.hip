#include "internal.h"
namespace trbl {
void tbme_gradient(const Model&, int, const double*, const double*, double*, double*, hipStream_t) {
  throw Error{TRBL_E_STATE, "gradient not built yet"};
}
}  // namespace trbl
