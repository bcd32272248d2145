// Fall-off / PLOG instantiations of the one-wavefront integrator and its
// single-call test kernels: the same source as integrate.hip, built as a
// translation unit of its own so that the two halves compile in parallel.
#define CHEM_INTEGRATE_PART 1
#include "integrate.hip"
