// Streaming kernel variants for float basis storage and the stencil operator.
#define FAB_PART_T float
#define FAB_PART_OP 0
#define FAB_PART_SUFFIX f32_stencil
#include "k_basis_part.inc"
