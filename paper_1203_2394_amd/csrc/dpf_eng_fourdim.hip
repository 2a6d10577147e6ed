// dpf_eng_fourdim.hip: step kernels of model 2 of Table 1 (2, 2, 1) for every tile class, and its engine table entry.
#include "dpf_engine_impl.hpp"

#include <math.h>

namespace dpf {

// Derived constants (computed in double, stored as float after the raw values).
static void derive_fourdim(const double* p, std::vector<float>& o) {
  const double qx1 = p[4], qx2 = p[5], qz1 = p[6], qz2 = p[7], cz = p[8], r = p[13];
  o.push_back((float)sqrt(qx1));                                          // sx1
  o.push_back((float)sqrt(qx2));                                          // sx2
  o.push_back((float)sqrt(qz1));                                          // sz1
  o.push_back((float)(cz / qz1));                                         // kz
  o.push_back((float)sqrt(qz2 - cz * cz / qz1));                          // szc
  o.push_back((float)(1.0 / qx1));                                        // inv_qx1
  o.push_back((float)(1.0 / qx2));                                        // inv_qx2
  o.push_back((float)(-0.5 * (log(2.0 * M_PI * qx1) + log(2.0 * M_PI * qx2))));  // cx
  o.push_back((float)(1.0 / r));                                          // inv_r
  o.push_back((float)(-0.5 * log(2.0 * M_PI * r)));                       // cy
}

const Engine kEngFourDim = make_engine<FourDim>([](const double* p, std::vector<float>& o) { derive_fourdim(p, o); });

}  // namespace dpf
