// The solve of precision form PrecMixedP (kernel sequences in solver_impl.h).
#include "solver_impl.h"

template int run_solve<PrecMixedP>(gcr_solver*);
template int apply_form<PrecMixedP>(gcr_solver*, int, int, const double*, double*);
