// The FP64 refinement with working sets of up to 16 complex unknowns (Newton
// systems of order 32: registers up to order 16, LDS beyond): the same kernel as
// polish.hip, run over the pixels whose 8-slot pass filled its working set above tol.
#define L1LS_POLISH_SUPP 16
#define polish_kernel polish_kernel_mid
#define polish_lds_bytes polish_lds_bytes_mid
#define launch_polish_table launch_polish_mid_table
#define polish_stack polish_stack_mid
#include "polish.hip"
