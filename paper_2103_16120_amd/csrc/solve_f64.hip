// The solve of precision form PrecF64 (kernel sequences in solver_impl.h).
#include "solver_impl.h"

template int run_solve<PrecF64>(gcr_solver*);
template int apply_form<PrecF64>(gcr_solver*, int, int, const double*, double*);
