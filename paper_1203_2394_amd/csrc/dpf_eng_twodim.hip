// dpf_eng_twodim.hip: step kernels of model 1 of Table 1 (1, 1, 1), x sampled
// first, for every tile class, and its engine table entry.
#include "dpf_engine_impl.hpp"

#include <math.h>

namespace dpf {

// Derived constants (computed in double, stored as float after the raw
// values): the outer variable here is x.
static void derive_twodim(const double* p, std::vector<float>& o) {
  const double qx = p[0], qz = p[1], cxz = p[2], r = p[7];
  o.push_back((float)sqrt(qx));                          // so
  o.push_back((float)(cxz / qx));                        // k
  o.push_back((float)sqrt(qz - cxz * cxz / qx));         // sic
  o.push_back((float)(1.0 / qx));                        // inv_qo
  o.push_back((float)(-0.5 * log(2.0 * M_PI * qx)));     // co
  o.push_back((float)(1.0 / r));                         // inv_r
  o.push_back((float)(-0.5 * log(2.0 * M_PI * r)));      // cy
}

const Engine kEngTwoDim = make_engine<TwoDim>([](const double* p, std::vector<float>& o) { derive_twodim(p, o); });

}  // namespace dpf
