// inc_bound_check.hip -- host entry points to the rounding bounds of the
// incremental ||A^T r||_inf (inc_bound.hpp), the very functions the kernels
// call, for the CPU tests of the bound (libpcdm_check.so; not part of the
// method's C ABI).
#include "inc_bound.hpp"

extern "C" {
double pcdm_check_inc_gamma(double dmax) { return pcdm::inc_gamma(dmax); }
double pcdm_check_inc_l1_factor(double dmax) { return pcdm::inc_l1_factor(dmax); }
double pcdm_check_inc_shift(double dlt, double rmax, double gam) { return pcdm::inc_shift(dlt, rmax, gam); }
double pcdm_check_inc_lower(double m_old, double nrm_max, double D) { return pcdm::inc_lower(m_old, nrm_max, D); }
double pcdm_check_inc_moved(double ub, double nrm, double D) { return pcdm::inc_moved(ub, nrm, D); }
}
