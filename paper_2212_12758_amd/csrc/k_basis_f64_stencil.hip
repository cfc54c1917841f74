// Streaming kernel variants for double basis storage and the stencil operator.
#define FAB_PART_T double
#define FAB_PART_OP 0
#define FAB_PART_SUFFIX f64_stencil
#include "k_basis_part.inc"
