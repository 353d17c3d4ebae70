// The solve of precision form PrecSingleD (kernel sequences in solver_impl.h).
#include "solver_impl.h"

template int run_solve<PrecSingleD>(gcr_solver*);
template int apply_form<PrecSingleD>(gcr_solver*, int, int, const double*, double*);
