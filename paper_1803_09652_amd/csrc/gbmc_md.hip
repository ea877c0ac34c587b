// Dynamics between Monte Carlo attempts: one leapfrog Langevin step
// (Loncharich, Brooks & Pastor, Biopolymers 32 (1992) 523), the thermostat of
// the implicit-solvent simulations (section III.D), driven by the forces of
// gb_energy_forces plus an optional harmonic restraint of every atom to
// reference coordinates.
//
// Memory-bound elementwise work: one thread per atom, every array read and
// written once (coalesced: caller order, x/y/z/v/xi/xref component-major,
// force [N][3]).  The update runs in FP64 whatever the storage precision.
#include "gbmc_internal.h"

namespace gbmc {

namespace {

// 1 kcal/mol per (amu Angstrom) in Angstrom/ps^2 (4184 J / (1e-3 kg 1e-10 m)
// = 4.184e16 m/s^2)
constexpr double kAccUnit = 418.4;

template <typename T>
__global__ __launch_bounds__(256) void k_md_langevin(int n, T* __restrict__ x, T* __restrict__ y,
                                                     T* __restrict__ z, T* __restrict__ v,
                                                     const T* __restrict__ force,
                                                     const T* __restrict__ inv_mass,
                                                     const T* __restrict__ xi,
                                                     const T* __restrict__ xref, double k_restr,
                                                     double dt, double c_old, double c_new,
                                                     double noise2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double im = (double)inv_mass[i];
    // per component: v' = c_new [c_old v + dt acc F / m + sig xi], x' = x + dt v'
    const double sig = sqrt(noise2 * im);
    const double kick = dt * kAccUnit * im;
    T* pos[3] = {x, y, z};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const size_t k = (size_t)c * n + i;
        const double p = (double)pos[c][i];
        double f = (double)force[3 * (size_t)i + c];
        if (xref) f -= k_restr * (p - (double)xref[k]);
        const double vn = c_new * (c_old * (double)v[k] + kick * f + sig * (double)xi[k]);
        v[k] = (T)vn;
        pos[c][i] = (T)(p + dt * vn);
    }
}

}  // namespace

template <typename T>
hipError_t launch_md_langevin(int n, T* x, T* y, T* z, T* v, const T* force, const T* inv_mass,
                              const T* xi, const T* xref, double k_restr, double dt, double gamma,
                              double T_kelvin, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const double a = 0.5 * gamma * dt;
    // sig^2 m = 2 gamma kB T dt (in A^2/ps^2 amu)
    const double noise2 = 2.0 * gamma * kKB * T_kelvin * dt * kAccUnit;
    hipLaunchKernelGGL(k_md_langevin<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, x, y, z, v,
                       force, inv_mass, xi, xref, k_restr, dt, 1.0 - a, 1.0 / (1.0 + a), noise2);
    return hipGetLastError();
}

template hipError_t launch_md_langevin<float>(int, float*, float*, float*, float*, const float*,
                                              const float*, const float*, const float*, double,
                                              double, double, double, hipStream_t);
template hipError_t launch_md_langevin<double>(int, double*, double*, double*, double*,
                                               const double*, const double*, const double*,
                                               const double*, double, double, double, double,
                                               hipStream_t);

}  // namespace gbmc
