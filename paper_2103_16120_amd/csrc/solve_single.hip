// The solve of precision form PrecSingle (kernel sequences in solver_impl.h).
#include "solver_impl.h"

template int run_solve<PrecSingle>(gcr_solver*);
template int apply_form<PrecSingle>(gcr_solver*, int, int, const double*, double*);
