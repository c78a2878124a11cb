// Encrypted CSR matrix-factorisation program.
#include "context.h"

namespace csrmf {

struct MfState {};

void destroy_mf(MfState* m) { delete m; }

}  // namespace csrmf
