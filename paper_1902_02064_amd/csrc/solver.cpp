#include "internal.h"
namespace trbl {
int solve(const Model&, const trbl_opts&, double*, void*, trbl_info*) {
  throw Error{TRBL_E_STATE, "solver not built yet"};
}
}  // namespace trbl
