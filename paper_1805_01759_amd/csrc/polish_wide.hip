// The FP64 refinement with working sets of up to 32 complex unknowns (Newton
// systems of order 64, factorised in LDS): the same kernel as polish.hip, run
// over the pixels whose 16-slot pass filled its working set above tol.
#define L1LS_POLISH_SUPP 32
#define polish_kernel polish_kernel_wide
#define polish_lds_bytes polish_lds_bytes_wide
#define launch_polish_table launch_polish_wide_table
#define polish_stack polish_stack_wide
#include "polish.hip"
