// dpf_eng_twodimz.hip: step kernels of model 1 of Table 1 (1, 1, 1), z sampled
// first, for every tile class, and its engine table entry.
#include "dpf_engine_impl.hpp"

#include <math.h>

namespace dpf {

// Derived constants (computed in double, stored as float after the raw
// values): the outer variable here is z.
static void derive_twodimz(const double* p, std::vector<float>& o) {
  const double qx = p[0], qz = p[1], cxz = p[2], r = p[7];
  o.push_back((float)sqrt(qz));                          // so
  o.push_back((float)(cxz / qz));                        // k
  o.push_back((float)sqrt(qx - cxz * cxz / qz));         // sic
  o.push_back((float)(1.0 / qz));                        // inv_qo
  o.push_back((float)(-0.5 * log(2.0 * M_PI * qz)));     // co
  o.push_back((float)(1.0 / r));                         // inv_r
  o.push_back((float)(-0.5 * log(2.0 * M_PI * r)));      // cy
}

const Engine kEngTwoDimZ = make_engine<TwoDimZ>([](const double* p, std::vector<float>& o) { derive_twodimz(p, o); });

}  // namespace dpf
