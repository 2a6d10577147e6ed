// dpf_eng_lingauss.hip: step kernels of the linear-Gaussian model (dx, dz, dy) = (1, 2, 1) for every tile class, and its engine table entry.
#include "dpf_engine_impl.hpp"

#include <math.h>

namespace dpf {

// Derived constants (computed in double, stored as float after the raw values).
static void derive_lingauss(int dx, int dz, int dy, const double* p, std::vector<float>& o) {
  const size_t iqx = dx * dx + dx * dz, iqz = iqx + 1 + dz * dz + dz * dx,
               ir = iqz + 1 + dy * dx + dy * dz;
  const double qx = p[iqx], qz = p[iqz], r = p[ir];
  o.push_back((float)sqrt(qx));
  o.push_back((float)sqrt(qz));
  o.push_back((float)(1.0 / qx));
  o.push_back((float)(1.0 / r));
  o.push_back((float)(-0.5 * dx * log(2.0 * M_PI * qx)));
  o.push_back((float)(-0.5 * dy * log(2.0 * M_PI * r)));
}

const Engine kEngLinGauss = make_engine<LinGauss<1, 2, 1>>([](const double* p, std::vector<float>& o) { derive_lingauss(1, 2, 1, p, o); });

}  // namespace dpf
