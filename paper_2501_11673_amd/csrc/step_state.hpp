// One block step's scalar bookkeeping on the device (Algorithms 2 and 5,
// Section 5.4), shared by the launch-per-phase projection kernels and the
// sparse team kernel: c for this step's momentum, ||r||^2 into the window
// sums E0 / E1, and at a checkpoint (the last step of each period of 2 zeta
// steps) the stop candidate and the revision of rho from the weighted average
// of window ratios (eq. (weighted)).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace kpp {

// rho = clamp(1 - r_hat^(1/zeta), 0, 1); no revision (0) when r_hat >= 1
__device__ __forceinline__ double state_rho_from_rate(double rhat, int zeta) {
  if (!(rhat < 1.0)) return 0.0;
  double r = 1.0 - pow(rhat, 1.0 / static_cast<double>(zeta));
  return fmin(1.0, fmax(0.0, r));
}

__device__ __forceinline__ void step_state_update(DevState& s, double rr, int32_t zeta, int32_t adaptive) {
  const double rho = s.rho;
  s.c = (1.0 - rho) / (1.0 + rho);
  const int64_t period = 2 * static_cast<int64_t>(zeta);
  const int64_t ph = s.t % period;
  if (ph < zeta)
    s.E0 += rr;
  else
    s.E1 += rr;
  if (ph == period - 1) {
    s.ckpts += 1;
    s.last_E1 = s.E1;
    s.rho_before = rho;
    s.cand = (s.E1 <= s.thr) ? 1 : 0;
    if (adaptive && s.E0 > 0.0) {
      const double q = s.E1 / s.E0;
      if (!s.have_rhat) {
        s.rhat = q;
        s.have_rhat = 1;
      } else {
        const double li = log(static_cast<double>(s.ckpt));
        const double li1 = log(static_cast<double>(s.ckpt) + 1.0);
        const double w = exp(li * li - li1 * li1);
        s.rhat = w * s.rhat + (1.0 - w) * q;
      }
      s.ckpt += 1;
      s.rho = state_rho_from_rate(s.rhat, zeta);
    }
    s.E0 = 0.0;
    s.E1 = 0.0;
  }
  s.t += 1;
}

}  // namespace kpp
