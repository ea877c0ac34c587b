// The plain FP64 GPU form of one full evaluation: the same Born radii,
// Coulomb + GB energies, forces (explicit and Born-chain), dE/dq and dE/drho
// as the batched passes, written the direct way: one thread per atom walks
// its whole row of the system (every ordered pair, as the definition sums
// them), closed forms with correctly rounded division, square root, exp and
// log, FP64 sums in a fixed order.  It is the reference point that the
// FP32-fixed form's pair rate is compared with, and needs no plan.
#include <hip/hip_runtime.h>

#include "gbmc_internal.h"

namespace gbmc {

namespace {

// kC = k / eps_in, kT = k (1/eps_in - 1/eps_out)
struct PlainConst {
    double alpha, beta, gamma, offset, kC, kT;
};

// System of atom i: the b with off[b] <= i < off[b + 1].
__device__ __forceinline__ int system_of(const int32_t* off, int B, int i)
{
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// HCT integral H(r; rt, S) (the part of ball j outside radius rt), closed form.
__device__ double plain_hct(double r, double rt, double S)
{
    const double U = r + S;
    if (rt >= U) return 0.0;
    const double L = fmax(rt, fabs(r - S));
    const double a = 1.0 / L, b = 1.0 / U;
    double H = 0.5 * (a - b + 0.25 * r * (b * b - a * a) + 0.5 / r * log(L / U)
                      + 0.25 * S * S / r * (a * a - b * b));
    if (rt < S - r) H += 1.0 / rt - a;
    return H;
}

// Its partials: d[0] = dH/dr, d[1] = dH/drt, d[2] = dH/dS.
__device__ void plain_hct_grad(double r, double rt, double S, double* d)
{
    d[0] = d[1] = d[2] = 0.0;
    const double U = r + S;
    if (rt >= U) return;
    double L = fabs(r - S);
    const bool l_rt = rt > L;
    if (l_rt) L = rt;
    const double a = 1.0 / L, b = 1.0 / U;
    d[0] = 0.5 * (0.25 * (b * b - a * a) * (1.0 + S * S / (r * r)) - log(L / U) / (2.0 * r * r));
    d[2] = 0.5 * S / (2.0 * r) * (a * a - b * b);
    if (l_rt)
        d[1] = 0.5 * ((L - r) * (L - r) - S * S) / (2.0 * r * L * L * L);
    else if (rt < S - r)
        d[1] = -1.0 / (rt * rt);
}

__device__ __forceinline__ double dist(const double* x, const double* y, const double* z, int i, int j,
                                       double& dx, double& dy, double& dz)
{
    dx = x[i] - x[j];
    dy = y[i] - y[j];
    dz = z[i] - z[j];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// Pass 1: descreening sum and OBC radius of atom i.
__global__ __launch_bounds__(256) void k_plain_radii(int N, int B, const int32_t* __restrict__ off,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ z,
                                                     const double* __restrict__ rho,
                                                     const double* __restrict__ scr, PlainConst c,
                                                     double* __restrict__ I_out,
                                                     double* __restrict__ R_out,
                                                     double* __restrict__ T_out,
                                                     double* __restrict__ dR_out,
                                                     double* __restrict__ born_R)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = system_of(off, B, i);
    const double rti = rho[i] - c.offset;
    double sum = 0.0;
    for (int j = off[b]; j < off[b + 1]; ++j) {
        if (j == i) continue;
        double dx, dy, dz;
        const double r = dist(x, y, z, i, j, dx, dy, dz);
        sum += plain_hct(r, rti, scr[j] * (rho[j] - c.offset));
    }
    const double psi = rti * sum;
    const double th = c.alpha * psi - c.beta * psi * psi + c.gamma * psi * psi * psi;
    const double t = tanh(th);
    const double R = 1.0 / (1.0 / rti - t / rho[i]);
    I_out[i] = sum;
    R_out[i] = R;
    T_out[i] = t;
    dR_out[i] = R * R * (1.0 - t * t) * (c.alpha - 2.0 * c.beta * psi + 3.0 * c.gamma * psi * psi) / rho[i];
    if (born_R) born_R[i] = R;
}

// Pass 2: the row of atom i: its energy shares (half of each pair's Coulomb
// term, all of its GB terms), explicit force, G = dE/dR and phi = dE/dq.
__global__ __launch_bounds__(256) void k_plain_energy(int N, int B, const int32_t* __restrict__ off,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ z,
                                                      const double* __restrict__ q,
                                                      const double* __restrict__ R, PlainConst c,
                                                      double* __restrict__ e_share,
                                                      double* __restrict__ F,
                                                      double* __restrict__ G,
                                                      double* __restrict__ phi)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = system_of(off, B, i);
    const double qi = q[i], Ri = R[i];
    double ec = 0.0, eg = qi * qi / Ri;
    double g = 0.5 * c.kT * qi * qi / (Ri * Ri);
    double ph = -c.kT * qi / Ri;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int j = off[b]; j < off[b + 1]; ++j) {
        if (j == i) continue;
        double dx, dy, dz;
        const double r = dist(x, y, z, i, j, dx, dy, dz);
        const double RR = Ri * R[j];
        const double D = r * r / (4.0 * RR);
        const double ex = exp(-D);
        const double f = sqrt(r * r + RR * ex);
        const double qq = qi * q[j];
        ec += 0.5 * qq / r;
        eg += qq / f;
        const double dfdr = r / f * (1.0 - 0.25 * ex);
        const double dEdr = -c.kC * qq / (r * r) + c.kT * qq / (f * f) * dfdr;
        fx -= dEdr * dx / r;
        fy -= dEdr * dy / r;
        fz -= dEdr * dz / r;
        g += c.kT * qq / (f * f) * (R[j] * ex * (1.0 + D) / (2.0 * f));
        ph += c.kC * q[j] / r - c.kT * q[j] / f;
    }
    e_share[i] = c.kC * ec;
    e_share[N + i] = -0.5 * c.kT * eg;
    F[i] = fx;
    F[N + i] = fy;
    F[2 * N + i] = fz;
    G[i] = g;
    phi[i] = ph;
}

// Pass 3: the Born-radius chain force on atom a and dE/drho_a, with
// B = G dR/dPsi of every atom of the row.
__global__ __launch_bounds__(256) void k_plain_chain(int N, int B, const int32_t* __restrict__ off,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ z,
                                                     const double* __restrict__ rho,
                                                     const double* __restrict__ scr,
                                                     const double* __restrict__ I,
                                                     const double* __restrict__ R,
                                                     const double* __restrict__ T,
                                                     const double* __restrict__ dR,
                                                     const double* __restrict__ G, PlainConst c,
                                                     const double* __restrict__ F,
                                                     const double* __restrict__ phi,
                                                     double* __restrict__ force,
                                                     double* __restrict__ dEdq,
                                                     double* __restrict__ dEdrho)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    const int b = system_of(off, B, a);
    const double rta = rho[a] - c.offset, Sa = scr[a] * rta;
    const double Ba = G[a] * dR[a];
    double fx = 0.0, fy = 0.0, fz = 0.0, drt = 0.0, dS = 0.0;
    for (int j = off[b]; j < off[b + 1]; ++j) {
        if (j == a) continue;
        double dx, dy, dz;
        const double r = dist(x, y, z, a, j, dx, dy, dz);
        const double rtj = rho[j] - c.offset;
        double gaj[3], gja[3];
        plain_hct_grad(r, rta, scr[j] * rtj, gaj);   // H(r_aj; rt_a, S_j) in Psi_a
        plain_hct_grad(r, rtj, Sa, gja);             // H(r_ja; rt_j, S_a) in Psi_j
        const double Bj = G[j] * dR[j];
        const double dEdr = Ba * rta * gaj[0] + Bj * rtj * gja[0];
        fx -= dEdr * dx / r;
        fy -= dEdr * dy / r;
        fz -= dEdr * dz / r;
        drt += gaj[1];
        dS += Bj * rtj * gja[2];
    }
    if (force) {
        force[3 * (size_t)a] = F[a] + fx;
        force[3 * (size_t)a + 1] = F[N + a] + fy;
        force[3 * (size_t)a + 2] = F[2 * N + a] + fz;
    }
    if (dEdq) dEdq[a] = phi[a];
    if (dEdrho)
        dEdrho[a] = G[a] * R[a] * R[a] * (1.0 / (rta * rta) - T[a] / (rho[a] * rho[a]))
                  + Ba * (I[a] + rta * drt) + scr[a] * dS;
}

// Per-system energies: one workgroup per system; each thread sums the shares
// of atoms tid, tid + 256, ... in index order, then a fixed tree over the 256
// partial sums (the same order on every run).
__global__ __launch_bounds__(256) void k_plain_energy_sum(int B, const int32_t* __restrict__ off,
                                                          int N,
                                                          const double* __restrict__ e_share,
                                                          double* __restrict__ e_coul,
                                                          double* __restrict__ e_gb)
{
    __shared__ double sc[256], sg[256];
    const int b = blockIdx.x, t = threadIdx.x;
    double ec = 0.0, eg = 0.0;
    for (int i = off[b] + t; i < off[b + 1]; i += 256) {
        ec += e_share[i];
        eg += e_share[N + i];
    }
    sc[t] = ec;
    sg[t] = eg;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            sc[t] += sc[t + h];
            sg[t] += sg[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (e_coul) e_coul[b] = sc[0];
        if (e_gb) e_gb[b] = sg[0];
    }
}

}  // namespace

size_t plain_workspace_bytes(int n_atoms)
{
    return sizeof(double) * (size_t)n_atoms * 12;
}

hipError_t launch_plain_fp64(int B, const int32_t* off, int N, const double* x, const double* y,
                             const double* z, const double* q, const double* rho,
                             const double* scr, const GBConst& gc, void* ws, double* born_R,
                             double* e_coul, double* e_gb, double* force, double* dEdq,
                             double* dEdrho, hipStream_t s)
{
    if (B == 0) return hipSuccess;
    double* w = static_cast<double*>(ws);
    double *I = w, *R = w + N, *T = w + 2 * (size_t)N, *dR = w + 3 * (size_t)N,
           *G = w + 4 * (size_t)N, *phi = w + 5 * (size_t)N, *es = w + 6 * (size_t)N,
           *F = w + 8 * (size_t)N;
    const PlainConst pc{gc.alpha, gc.beta, gc.gamma, gc.offset, gc.kC, gc.kT};
    const int nb = (N + 255) / 256;
    if (N > 0) {
        hipLaunchKernelGGL(k_plain_radii, dim3(nb), dim3(256), 0, s, N, B, off, x, y, z, rho, scr, pc,
                           I, R, T, dR, born_R);
        hipLaunchKernelGGL(k_plain_energy, dim3(nb), dim3(256), 0, s, N, B, off, x, y, z, q, R, pc,
                           es, F, G, phi);
        hipLaunchKernelGGL(k_plain_chain, dim3(nb), dim3(256), 0, s, N, B, off, x, y, z, rho, scr, I,
                           R, T, dR, G, pc, F, phi, force, dEdq, dEdrho);
    }
    hipLaunchKernelGGL(k_plain_energy_sum, dim3(B), dim3(256), 0, s, B, off, N, es, e_coul, e_gb);
    return hipGetLastError();
}

}  // namespace gbmc
