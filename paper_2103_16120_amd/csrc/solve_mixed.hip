// The solve of precision form PrecMixed (kernel sequences in solver_impl.h).
#include "solver_impl.h"

template int run_solve<PrecMixed>(gcr_solver*);
template int apply_form<PrecMixed>(gcr_solver*, int, int, const double*, double*);
