// The solve of precision form PrecMixedD (kernel sequences in solver_impl.h).
#include "solver_impl.h"

template int run_solve<PrecMixedD>(gcr_solver*);
template int apply_form<PrecMixedD>(gcr_solver*, int, int, const double*, double*);
