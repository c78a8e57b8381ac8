// Entry points whose solvers are not built yet report PN_ERR_UNSUPPORTED.
#include "pn_solvers.hpp"

namespace pn {

}  // namespace pn
