// Inertial / diffusive particle step (Sec. 4.3: inertial particles and
// high-diffusivity markers can move more than one grid spacing per step).
// Stokes drag dx/dt = v, dv/dt = (u(x) - v)/tau over a step h, solved exactly
// with the fluid velocity along the step taken as linear in time between
// u0 = u(x) and u1 = u(x*), x* being where the exact solution ends if the
// fluid velocity stays u0; d is an optional displacement increment (a
// diffusive marker's random step), added to the predictor and kept:
//   x* = x + cv v + cu u0 + d,   x+ = x* + cc (u1 - u0),
//   v+ = E v + bu0 u0 + b u1,
// with r = h/tau, E = e^-r, p1 = (1 - E)/r, p2 = (1 - p1)/r:
//   cv = h p1, cu = h (1 - p1), cc = h (1/2 - p2), b = 1 - p1, bu0 = p1 - E.
// tau = 0 (the fluid tracer) is the limit cv = 0, cu = h, cc = h/2, E = 0,
// bu0 = 0, b = 1: Heun's step.  All in FP64; the coefficients are formed
// once per call on the host.
#pragma once

namespace pt {

struct InertialCoef {
  double cv, cu, cc, E, bu0, b;
};

__device__ __forceinline__ double inertial_predict(const InertialCoef& k, double x, double v,
                                                   double u0, double d) {
  return x + k.cv * v + k.cu * u0 + d;
}

__device__ __forceinline__ double inertial_correct(const InertialCoef& k, double xs, double u0,
                                                   double u1) {
  return xs + k.cc * (u1 - u0);
}

__device__ __forceinline__ double inertial_velocity(const InertialCoef& k, double v, double u0,
                                                    double u1) {
  return k.E * v + k.bu0 * u0 + k.b * u1;
}

// Host: the coefficients for a step h > 0 and a response time tau >= 0.
InertialCoef inertial_coef(double h, double tau);

}  // namespace pt
