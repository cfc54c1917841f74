// Streaming kernel variants for float basis storage and the csr operator.
#define FAB_PART_T float
#define FAB_PART_OP 1
#define FAB_PART_SUFFIX f32_csr
#include "k_basis_part.inc"
