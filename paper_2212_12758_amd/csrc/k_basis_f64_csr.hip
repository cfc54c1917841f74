// Streaming kernel variants for double basis storage and the csr operator.
#define FAB_PART_T double
#define FAB_PART_OP 1
#define FAB_PART_SUFFIX f64_csr
#include "k_basis_part.inc"
