// gbmc_kernels.hip -- HIP kernels for gfx950 (CDNA4): all-pairs GB-OBC radii,
// energy and forces, FP64 Monte Carlo Delta E / Delta G, the Metropolis step and
// the E-REMD exchange.
//
// Pair work is split into 64 x 64 tiles of one system (i block I, j block J,
// J >= I); one wavefront owns a tile and evaluates every unordered pair of it
// once.  Lane l keeps atom i = 64 I + l and its i-side sums in registers.  The
// j block is staged twice into the wavefront's LDS slice, so that at step k
// lane l reads j = (l + k) mod 64 from slot l + k without a wrap.  The j-side
// sums live in registers too: lane l holds the sums of the j it visits, and
// after every step they move one lane down with a DPP full-wavefront rotation
// (wave_rol:1, lane l <- lane l + 1), so at step k + 1 each lane again holds
// the sums of the j it is about to visit.  After the 64 steps of a tile every
// lane holds the sums of j = 64 J + l.  (LDS float atomics for the j side were
// measured ~40x slower than this rotation on gfx950.)
//
// At the end of a tile both partial sums are rounded once into 64-bit fixed
// point; tiles combine with integer atomics, so sums are exact, the result does
// not depend on the order in which tiles run, and it does not depend on how
// many j blocks one work item walks.
//
// Atoms past the end of a system (ragged last block) are dummies with q = 0,
// screen = 0, B = 0 placed far away: every pair term involving a dummy vanishes
// on the real atom's side, and dummies are never flushed.

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "gbmc_internal.h"

namespace gbmc {

#include "hct_poly.inc"

constexpr double kLn2 = 0.693147180559945309;
constexpr double kLog2e = 1.44269504088896340736;
constexpr double kLn10 = 2.302585092994045684;
// sqrt(log2(e) / 4): a_i a_j r^2 = r^2 log2(e) / (4 R_i R_j)
constexpr double kAScale = 0.60056120439322491;

// ------------------------------------------------------------------ math

__device__ __forceinline__ float rsq(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ float exp2neg(float t) { return __builtin_amdgcn_exp2f(-t); }
// FP64 1/sqrt and 1/x: hardware estimates refined by two Newton steps (within
// an ulp or two of the rounded result, at a fraction of the cost of the
// correctly rounded division and square root).
__device__ __forceinline__ double rsq64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}
__device__ __forceinline__ double rcp64(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    y = fma(y, fma(-x, y, 1.0), y);
    return y;
}
__device__ __forceinline__ double rsq(double v) { return rsq64(v); }
__device__ __forceinline__ double rcp(double v) { return rcp64(v); }
__device__ __forceinline__ double exp2neg(double t) { return exp2(-t); }

// 1/a and 1/b from one reciprocal: c = 1/(a b), 1/a = c b, 1/b = c a (a
// transcendental costs several ordinary instructions).  For the polynomial
// forms of the chain pass, where a, b = 1 - y >= 0.6 for every pair whose terms
// are kept.
__device__ __forceinline__ void rcp_pair(float a, float b, float& ia, float& ib)
{
    const float c = rcp(a * b);
    ia = c * b;
    ib = c * a;
}
__device__ __forceinline__ void rcp_pair(double a, double b, double& ia, double& ib)
{
    const double c = rcp64(a * b);
    ia = c * b;
    ib = c * a;
}

// Fixed-point value of v; an out-of-range (or NaN) v gives 0 and sets bad.
// The flag stays in a register until the work item ends, so that the pair
// loops issue no conditional stores.
__device__ __forceinline__ long long to_fixed(double v, double scale, bool& bad)
{
    double s = v * scale;
    const bool ok = fabs(s) < kFixLimit;
    bad |= !ok;
    return ok ? __double2ll_rn(s) : 0ll;
}

// The same for an FP32 value in FP32 arithmetic, with the same result: with
// m = |v| scale / 2^32 (exact, scale is a power of two), h = floor(m) and the
// fraction m - h (exact for m >= 0), the nearest integer to |v| scale is
// h 2^32 + rint((m - h) 2^32) (h 2^32 is even, so ties go the same way), and
// rint(-x) = -rint(x).
__device__ __forceinline__ long long to_fixed(float v, double scale, bool& bad)
{
    const float a = v * (float)(scale * (1.0 / 4294967296.0));
    const float m = fabsf(a);
    const bool ok = m < 1073741824.0f;                  // |v scale| < 2^62
    bad |= !ok;
    const float h = floorf(m);
    const float lo = __builtin_rintf((m - h) * 4294967296.0f);
    const long long r = (long long)(((unsigned long long)(unsigned)h << 32) | (unsigned)lo);
    return ok ? (a < 0.0f ? -r : r) : 0ll;
}

// Row of atom a in a system of n >= 1 atoms.  Lanes past the end read (and add
// zero to) the atom a mod n, so every lane issues the same memory operations
// (the wait for the next block's loads then does not depend on the lane mix)
// and the zero additions of one block go to distinct addresses.
__device__ __forceinline__ int clamp_atom(int a, int n) { return a < n ? a : a % n; }

__device__ __forceinline__ void fx_add(unsigned long long* p, long long v)
{
    atomicAdd(p, (unsigned long long)v);
}

// Per-atom values that one wave of a queued launch writes and other waves
// of the same launch read (Born radii, dR/dPsi and G sums of finished blocks)
// move through device-scope loads and stores (sc1: coherent across the L2
// caches of the XCDs, which plain loads are not within one launch).
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p)
{
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// --------------------------------------------------- cross-lane movement
// rot1: lane l receives lane (l + 1) mod 64 (DPP wave_rol:1, all lanes active).
__device__ __forceinline__ int rot1i(int v)
{
    // old == src: the move happens in place, with no extra register copies
    return __builtin_amdgcn_update_dpp(v, v, 0x134, 0xF, 0xF, false);
}
__device__ __forceinline__ float rot1(float v)
{
    return __builtin_bit_cast(float, rot1i(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double rot1(double v)
{
    long long b = __builtin_bit_cast(long long, v);
    int lo = rot1i((int)b), hi = rot1i((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// lane l receives the value of lane src (ds_bpermute; LDS crossbar, no LDS memory)
__device__ __forceinline__ int from_lane_i(int v, int src)
{
    return __builtin_amdgcn_ds_bpermute(src << 2, v);
}
__device__ __forceinline__ float from_lane(float v, int src)
{
    return __builtin_bit_cast(float, from_lane_i(__builtin_bit_cast(int, v), src));
}
__device__ __forceinline__ double from_lane(double v, int src)
{
    long long b = __builtin_bit_cast(long long, v);
    int lo = from_lane_i((int)b, src), hi = from_lane_i((int)(b >> 32), src);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// ------------------------------------------------------------ HCT integral
// H(r; rt, S): the (1/4 pi) integral of |x|^-4 over the part of the ball of
// radius S at distance r outside radius rt.  General closed form (all cases),
// used by the FP64 plans.
__device__ __forceinline__ double hct_general(double r, double invr, double rt, double S)
{
    double U = r + S;
    double L = fmax(rt, fabs(r - S));
    double a = 1.0 / L, b = 1.0 / U;
    double a2 = a * a, b2 = b * b;
    double h = (a - b) + 0.25 * r * (b2 - a2) + 0.5 * invr * log(L * b) + 0.25 * S * S * invr * (a2 - b2);
    double H = 0.5 * h;
    if (rt < S - r) H += 1.0 / rt - a;
    return rt >= U ? 0.0 : H;
}

// Partials of H: dH/dr, dH/drt, dH/dS (all cases; FP64).  dh/dL vanishes at
// L = r - S, dh/dU at U = r + S, and in the engulfed case the L-dependence
// cancels against the full-shell term, so dr and dS are partials at fixed L, U.
__device__ __forceinline__ void hct_general_grad(double r, double invr, double rt, double S,
                                                 double& dr, double& drt, double& dS)
{
    double U = r + S;
    double ad = fabs(r - S);
    bool l_rt = rt > ad;
    double L = l_rt ? rt : ad;
    double a = 1.0 / L, b = 1.0 / U;
    double a2 = a * a, b2 = b * b;
    double invr2 = invr * invr;
    dr = 0.5 * (0.25 * (b2 - a2) * (1.0 + S * S * invr2) - 0.5 * log(L * b) * invr2);
    dS = 0.25 * S * invr * (a2 - b2);
    drt = l_rt ? 0.25 * ((L - r) * (L - r) - S * S) * invr * a2 * a
               : (rt < S - r ? -1.0 / (rt * rt) : 0.0);
    if (rt >= U) { dr = 0.0; drt = 0.0; dS = 0.0; }
}

// FP32 form of H and its partials that does not cancel when the spheres
// overlap.  With L = max(rt, |r - S|), U = r + S, e = (U - L)/L:
//   (1/(4r)) * integral_L^U (S^2 - (t - r)^2) / t^3 dt = J / (4r),
//   J = [e - log(1 + e)] + (S - r) e^2 / (2U),
// and, at fixed L (the L-dependence vanishes or cancels, see hct_general_grad),
//   dJ/dr = e/U - e^2/(2U) + (S - r)(e/(L U) - e^2/(2U^2)),
//   dJ/dS = e/U + e^2/(2U) + (S - r)(e/(L U) - e^2/(2U^2)),
//   dH/drt = -e (L + S - r) / (4 r L^2) when L = rt.
// e - log(1 + e) = e z - 2 z^3 (1/3 + z^2/5 + ...), z = e / (2 + e), for e <= 1.
__device__ __forceinline__ float e_minus_log1p(float e)
{
    if (e <= 1.0f) {
        float z = e * rcp(2.0f + e), z2 = z * z;
        float p = 1.0f / 17.0f;
        p = fmaf(p, z2, 1.0f / 15.0f);
        p = fmaf(p, z2, 1.0f / 13.0f);
        p = fmaf(p, z2, 1.0f / 11.0f);
        p = fmaf(p, z2, 1.0f / 9.0f);
        p = fmaf(p, z2, 1.0f / 7.0f);
        p = fmaf(p, z2, 1.0f / 5.0f);
        p = fmaf(p, z2, 1.0f / 3.0f);
        return fmaf(-2.0f * z * z2, p, e * z);
    }
    return e - __builtin_amdgcn_logf(1.0f + e) * 0.693147180559945309f;
}

template <bool GRAD>
__device__ __forceinline__ float hct_slow32(float r, float invr, float rt, float S, float* g)
{
    float U = r + S;
    float dRS = r - S, ad = fabsf(dRS);
    bool l_rt = rt > ad;
    float L = l_rt ? rt : ad;
    float delta = l_rt ? ((S - rt) + r) : (dRS < 0.0f ? 2.0f * r : 2.0f * S);   // U - L
    float invL = rcp(L), invU = rcp(U);
    float e = delta * invL;
    float J = fmaf((S - r) * 0.5f * invU, e * e, e_minus_log1p(e));
    float H = 0.25f * invr * J;
    bool eng = rt < S - r;
    if (eng) H += ((S - rt) - r) * invL * rcp(rt);   // 1/rt - 1/L
    bool zero = rt >= U;
    if (GRAD) {
        float eU = e * invU;
        float cross = (S - r) * eU * (invL - 0.5f * e * invU);
        float Jr = eU * (1.0f - 0.5f * e) + cross;
        float JS = eU * (1.0f + 0.5f * e) + cross;
        float irt = rcp(rt);
        g[0] = zero ? 0.0f : 0.25f * invr * (Jr - J * invr);
        g[1] = zero ? 0.0f : (l_rt ? -0.25f * invr * e * (L + S - r) * invL * invL : (eng ? -irt * irt : 0.0f));
        g[2] = zero ? 0.0f : 0.25f * invr * JS;
    }
    return zero ? 0.0f : H;
}

__device__ __forceinline__ void dist64(double xi, double yi, double zi, double xj, double yj,
                                       double zj, double& r, double& invr)
{
    double dx = xi - xj, dy = yi - yj, dz = zi - zj;
    double r2 = dx * dx + dy * dy + dz * dz;
    invr = rsq64(r2);
    r = r2 * invr;
}

// Pass-1 pair: H(r; rt_i, S_j) and H(r; rt_j, S_i).
// FP32: non-overlapping pairs (r - S >= rt, x = S/r with x^2 <= YMAX) use
// H = x^3 P(x^2) / r; every other pair takes hct_slow32.
__device__ __forceinline__ void radii_pair(float xi, float yi, float zi, float xj, float yj, float zj,
                                           float rti, float Si, float rtj, float Sj, float& hij,
                                           float& hji)
{
    float dx = xi - xj, dy = yi - yj, dz = zi - zj;
    float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    float invr = rsq(r2);
    float r = r2 * invr;
    float xij = Sj * invr, yij = xij * xij;
    float xji = Si * invr, yji = xji * xji;
    hij = xij * yij * invr * hct_poly(yij);
    hji = xji * yji * invr * hct_poly(yji);
    bool f_ij = (r - Sj >= rti) & (yij <= GBMC_HCT_YMAX);
    bool f_ji = (r - Si >= rtj) & (yji <= GBMC_HCT_YMAX);
    if (!(f_ij & f_ji)) {
        if (!f_ij) hij = hct_slow32<false>(r, invr, rti, Sj, nullptr);
        if (!f_ji) hji = hct_slow32<false>(r, invr, rtj, Si, nullptr);
    }
}

// The polynomial form alone, for walks that defer the pairs it does not cover
// (as chain_pair_fast): a pair that needs the closed form in either direction
// gets zero terms and, if act, its bit in mask.
template <bool TEST = true>
__device__ __forceinline__ void radii_pair_fast(float xi, float yi, float zi, float xj, float yj,
                                                float zj, float rti, float Si, float rtj, float Sj,
                                                bool act, unsigned long long bit, float& hij,
                                                float& hji, unsigned long long& mask)
{
    float dx = xi - xj, dy = yi - yj, dz = zi - zj;
    float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    float invr = rsq(r2);
    float r = r2 * invr;
    float xij = Sj * invr, yij = xij * xij;
    float xji = Si * invr, yji = xji * xji;
    // a separated tile (!TEST): every pair is non-overlapping with y <= YFAR,
    // where the short fit is as accurate as the wide one
    hij = xij * yij * invr * (TEST ? hct_poly(yij) : hct_poly_far(yij));
    hji = xji * yji * invr * (TEST ? hct_poly(yji) : hct_poly_far(yji));
    if constexpr (!TEST) return;
    const bool fast = (r - Sj >= rti) & (yij <= GBMC_HCT_YMAX) & (r - Si >= rtj) &
                      (yji <= GBMC_HCT_YMAX);
    if (__builtin_amdgcn_ballot_w64(!fast) != 0ull) {
        asm volatile("");                       // keeps this a branch
        hij = fast ? hij : 0.0f;
        hji = fast ? hji : 0.0f;
        mask |= (!fast && act) ? bit : 0ull;
    }
}

// FP64: the same split, with a degree-14 polynomial on y <= 0.25 (one ulp);
// every other pair takes the closed form.
__device__ __forceinline__ void radii_pair(double xi, double yi, double zi, double xj, double yj,
                                           double zj, double rti, double Si, double rtj, double Sj,
                                           double& hij, double& hji)
{
    double r, invr;
    dist64(xi, yi, zi, xj, yj, zj, r, invr);
    const double xij = Sj * invr, yij = xij * xij;
    const double xji = Si * invr, yji = xji * xji;
    hij = xij * yij * invr * hct_poly64(yij);
    hji = xji * yji * invr * hct_poly64(yji);
    const bool f_ij = (r - Sj >= rti) & (yij <= GBMC_HCT_YMAX64);
    const bool f_ji = (r - Si >= rtj) & (yji <= GBMC_HCT_YMAX64);
    if (!(f_ij & f_ji)) {
        if (!f_ij) hij = hct_general(r, invr, rti, Sj);
        if (!f_ji) hji = hct_general(r, invr, rtj, Si);
    }
}

// Pass-3 pair terms with the Born chain weights bi = B_i rt_i, bj = B_j rt_j
// applied: dEdr = bi dH(r; rt_i, S_j)/dr + bj dH(r; rt_j, S_i)/dr, the S
// derivatives gij2 = dH(r; rt_i, S_j)/dS and gji2 = dH(r; rt_j, S_i)/dS, and
// the rt derivatives, nonzero only for overlapping pairs, added as
// dri += bi dH(r; rt_i, S_j)/drt and drj += bj dH(r; rt_j, S_i)/drt.
// FP32: non-overlapping directions use the polynomial form,
//   dH/dr = -x^3 (P + (1 - y)^-2) / r^2,  dH/dS = y (1 - y)^-2 / r^2,
// with the common 1/r^2 of the two dH/dr applied once.
__device__ __forceinline__ void chain_pair(float r, float r2, float invr, float rti, float Si,
                                           float rtj, float Sj, float bi, float bj, float& dEdr,
                                           float& gij2, float& gji2, float& dri, float& drj)
{
    const float u = invr * invr;
    const float xij = Sj * invr, yij = xij * xij;
    const float xji = Si * invr, yji = xji * xji;
    float wij = rcp(1.0f - yij), wji = rcp(1.0f - yji);
    wij *= wij;
    wji *= wji;
    // -r^2 dH/dr = x^3 (P + w) = x (y P + t), r^2 dH/dS = t = y w
    const float tij = yij * wij, tji = yji * wji;
    float aij = xij * fmaf(yij, hct_poly_d(yij), tij);
    float aji = xji * fmaf(yji, hct_poly_d(yji), tji);
    gij2 = tij * u;
    gji2 = tji * u;
    const bool f_ij = (r - Sj >= rti) & (yij <= GBMC_HCT_YMAX);
    const bool f_ji = (r - Si >= rtj) & (yji <= GBMC_HCT_YMAX);
    if (!(f_ij & f_ji)) {
        float g[3];
        if (!f_ij) {
            hct_slow32<true>(r, invr, rti, Sj, g);
            aij = -g[0] * r2;
            gij2 = g[2];
            dri = fmaf(bi, g[1], dri);
        }
        if (!f_ji) {
            hct_slow32<true>(r, invr, rtj, Si, g);
            aji = -g[0] * r2;
            gji2 = g[2];
            drj = fmaf(bj, g[1], drj);
        }
    }
    dEdr = -u * fmaf(bi, aij, bj * aji);
}

// The polynomial form alone, for walks that defer the pairs it does not cover.
// A pair that needs the closed form in either direction (act only) gets zero
// terms and its bit in mask (one wave-uniform branch, taken only in the steps
// that meet such a pair); the caller evaluates those pairs after the walk.
// On separated tiles (TEST false, y <= YFAR) the factor (1 - y)^-2 comes from
// its degree-5 fit, without a reciprocal.
template <bool TEST = true>
__device__ __forceinline__ void chain_pair_fast(float r, float invr, float rti, float Si, float rtj,
                                                float Sj, float bi, float bj, bool act,
                                                unsigned long long bit, float& dEdr, float& gij2,
                                                float& gji2, unsigned long long& mask)
{
    const float u = invr * invr;
    const float xij = Sj * invr, yij = xij * xij;
    const float xji = Si * invr, yji = xji * xji;
    float wij, wji;
    if constexpr (TEST) {
        rcp_pair(1.0f - yij, 1.0f - yji, wij, wji);
        wij *= wij;
        wji *= wji;
    } else {
        wij = hct_w_far(yij);
        wji = hct_w_far(yji);
    }
    const float tij = yij * wij, tji = yji * wji;
    float aij = xij * fmaf(yij, TEST ? hct_poly_d(yij) : hct_poly_far(yij), tij);
    float aji = xji * fmaf(yji, TEST ? hct_poly_d(yji) : hct_poly_far(yji), tji);
    gij2 = tij * u;
    gji2 = tji * u;
    const bool fast = !TEST || ((r - Sj >= rti) & (yij <= GBMC_HCT_YMAX) & (r - Si >= rtj) &
                                (yji <= GBMC_HCT_YMAX));
    if (TEST && __builtin_amdgcn_ballot_w64(!fast) != 0ull) {
        // an empty volatile statement keeps this a branch (not selects on
        // every step)
        asm volatile("");
        aij = fast ? aij : 0.0f;
        aji = fast ? aji : 0.0f;
        gij2 = fast ? gij2 : 0.0f;
        gji2 = fast ? gji2 : 0.0f;
        mask |= (!fast && act) ? bit : 0ull;
    }
    dEdr = -u * fmaf(bi, aij, bj * aji);
}

// FP64: the same split with the FP64 polynomial; overlapping pairs take the
// closed-form partials.
__device__ __forceinline__ void chain_pair(double r, double r2, double invr, double rti, double Si,
                                           double rtj, double Sj, double bi, double bj,
                                           double& dEdr, double& gij2, double& gji2, double& dri,
                                           double& drj)
{
    const double u = invr * invr;
    const double xij = Sj * invr, yij = xij * xij;
    const double xji = Si * invr, yji = xji * xji;
    double wij = rcp64(1.0 - yij), wji = rcp64(1.0 - yji);
    wij *= wij;
    wji *= wji;
    double aij = xij * yij * (hct_poly64(yij) + wij);    // -r^2 dH/dr
    double aji = xji * yji * (hct_poly64(yji) + wji);
    gij2 = yij * wij * u;
    gji2 = yji * wji * u;
    const bool f_ij = (r - Sj >= rti) & (yij <= GBMC_HCT_YMAX64);
    const bool f_ji = (r - Si >= rtj) & (yji <= GBMC_HCT_YMAX64);
    if (!(f_ij & f_ji)) {
        double g0, g1, g2;
        if (!f_ij) {
            hct_general_grad(r, invr, rti, Sj, g0, g1, g2);
            aij = -g0 * r2;
            gij2 = g2;
            dri = fma(bi, g1, dri);
        }
        if (!f_ji) {
            hct_general_grad(r, invr, rtj, Si, g0, g1, g2);
            aji = -g0 * r2;
            gji2 = g2;
            drj = fma(bj, g1, drj);
        }
    }
    dEdr = -u * fma(bi, aij, bj * aji);
}

// FP64 forms of the two deferring pair functions (polynomial of degree 14 on
// y <= 0.25; the pairs outside it are marked, as in FP32).
template <bool TEST = true>
__device__ __forceinline__ void radii_pair_fast(double xi, double yi, double zi, double xj,
                                                double yj, double zj, double rti, double Si,
                                                double rtj, double Sj, bool act,
                                                unsigned long long bit, double& hij, double& hji,
                                                unsigned long long& mask)
{
    double r, invr;
    dist64(xi, yi, zi, xj, yj, zj, r, invr);
    const double xij = Sj * invr, yij = xij * xij;
    const double xji = Si * invr, yji = xji * xji;
    hij = xij * yij * invr * (TEST ? hct_poly64(yij) : hct_poly64_far(yij));
    hji = xji * yji * invr * (TEST ? hct_poly64(yji) : hct_poly64_far(yji));
    if constexpr (!TEST) return;
    const bool fast = (r - Sj >= rti) & (yij <= GBMC_HCT_YMAX64) & (r - Si >= rtj) &
                      (yji <= GBMC_HCT_YMAX64);
    if (__builtin_amdgcn_ballot_w64(!fast) != 0ull) {
        asm volatile("");                       // keeps this a branch
        hij = fast ? hij : 0.0;
        hji = fast ? hji : 0.0;
        mask |= (!fast && act) ? bit : 0ull;
    }
}

template <bool TEST = true>
__device__ __forceinline__ void chain_pair_fast(double r, double invr, double rti, double Si,
                                                double rtj, double Sj, double bi, double bj,
                                                bool act, unsigned long long bit, double& dEdr,
                                                double& gij2, double& gji2,
                                                unsigned long long& mask)
{
    const double u = invr * invr;
    const double xij = Sj * invr, yij = xij * xij;
    const double xji = Si * invr, yji = xji * xji;
    double wij, wji;
    rcp_pair(1.0 - yij, 1.0 - yji, wij, wji);
    wij *= wij;
    wji *= wji;
    double aij = xij * yij * ((TEST ? hct_poly64(yij) : hct_poly64_far(yij)) + wij);   // -r^2 dH/dr
    double aji = xji * yji * ((TEST ? hct_poly64(yji) : hct_poly64_far(yji)) + wji);
    gij2 = yij * wij * u;
    gji2 = yji * wji * u;
    const bool fast = !TEST || ((r - Sj >= rti) & (yij <= GBMC_HCT_YMAX64) & (r - Si >= rtj) &
                                (yji <= GBMC_HCT_YMAX64));
    if (TEST && __builtin_amdgcn_ballot_w64(!fast) != 0ull) {
        asm volatile("");
        aij = fast ? aij : 0.0;
        aji = fast ? aji : 0.0;
        gij2 = fast ? gij2 : 0.0;
        gji2 = fast ? gji2 : 0.0;
        mask |= (!fast && act) ? bit : 0ull;
    }
    dEdr = -u * fma(bi, aij, bj * aji);
}

// The closed form of H and of its partials (dH/dr, dH/drt, dH/dS) in either
// precision, for the deferred pairs.
__device__ __forceinline__ float slow_H(float r, float invr, float rt, float S)
{
    return hct_slow32<false>(r, invr, rt, S, nullptr);
}
__device__ __forceinline__ double slow_H(double r, double invr, double rt, double S)
{
    return hct_general(r, invr, rt, S);
}
__device__ __forceinline__ void slow_grad(float r, float invr, float rt, float S, float* g)
{
    hct_slow32<true>(r, invr, rt, S, g);
}
__device__ __forceinline__ void slow_grad(double r, double invr, double rt, double S, double* g)
{
    hct_general_grad(r, invr, rt, S, g[0], g[1], g[2]);
}

// ------------------------------------------------------- cutoff variants
// With the descreening cutoff c the integral is restricted to the sphere of
// radius c around atom i: H_c = H(r; rt, S) - H(r; c, S) for a ball j that
// straddles that sphere (r - S < c < r + S), H for a ball inside it, 0 for
// one beyond it (r - S >= c) or when c <= rt.  Straddling balls take the
// closed form for both terms.
__device__ __forceinline__ void radii_pair_cut(float xi, float yi, float zi, float xj, float yj,
                                               float zj, float rti, float Si, float rtj, float Sj,
                                               float c, float& hij, float& hji)
{
    float dx = xi - xj, dy = yi - yj, dz = zi - zj;
    float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    float invr = rsq(r2);
    float r = r2 * invr;
    float xij = Sj * invr, yij = xij * xij;
    float xji = Si * invr, yji = xji * xji;
    hij = xij * yij * invr * hct_poly(yij);
    hji = xji * yji * invr * hct_poly(yji);
    const bool out_ij = (r - Sj >= c) | (c <= rti), out_ji = (r - Si >= c) | (c <= rtj);
    const bool st_ij = !out_ij & (r + Sj > c), st_ji = !out_ji & (r + Si > c);
    const bool f_ij = (r - Sj >= rti) & (yij <= GBMC_HCT_YMAX);
    const bool f_ji = (r - Si >= rtj) & (yji <= GBMC_HCT_YMAX);
    if (!(f_ij & f_ji)) {
        if (!f_ij) hij = hct_slow32<false>(r, invr, rti, Sj, nullptr);
        if (!f_ji) hji = hct_slow32<false>(r, invr, rtj, Si, nullptr);
    }
    // the part of a straddling ball beyond c (the c term has L = c)
    if (st_ij | st_ji) {
        if (st_ij) hij -= hct_slow32<false>(r, invr, c, Sj, nullptr);
        if (st_ji) hji -= hct_slow32<false>(r, invr, c, Si, nullptr);
    }
    hij = out_ij ? 0.0f : hij;
    hji = out_ji ? 0.0f : hji;
}

__device__ __forceinline__ void radii_pair_cut(double xi, double yi, double zi, double xj,
                                               double yj, double zj, double rti, double Si,
                                               double rtj, double Sj, double c, double& hij,
                                               double& hji)
{
    double r, invr;
    dist64(xi, yi, zi, xj, yj, zj, r, invr);
    const double xij = Sj * invr, yij = xij * xij;
    const double xji = Si * invr, yji = xji * xji;
    hij = xij * yij * invr * hct_poly64(yij);
    hji = xji * yji * invr * hct_poly64(yji);
    const bool out_ij = (r - Sj >= c) | (c <= rti), out_ji = (r - Si >= c) | (c <= rtj);
    const bool st_ij = !out_ij & (r + Sj > c), st_ji = !out_ji & (r + Si > c);
    const bool f_ij = (r - Sj >= rti) & (yij <= GBMC_HCT_YMAX64);
    const bool f_ji = (r - Si >= rtj) & (yji <= GBMC_HCT_YMAX64);
    if (!(f_ij & f_ji)) {
        if (!f_ij) hij = hct_general(r, invr, rti, Sj);
        if (!f_ji) hji = hct_general(r, invr, rtj, Si);
    }
    if (st_ij | st_ji) {
        if (st_ij) hij -= hct_general(r, invr, c, Sj);
        if (st_ji) hji -= hct_general(r, invr, c, Si);
    }
    hij = out_ij ? 0.0 : hij;
    hji = out_ji ? 0.0 : hji;
}

// Pass-3 pair terms of H_c (see chain_pair): the c term contributes to the r
// and S partials, not to the rt partial.
__device__ __forceinline__ void chain_pair_cut(float r, float r2, float invr, float rti, float Si,
                                               float rtj, float Sj, float bi, float bj, float c,
                                               float& dEdr, float& gij2, float& gji2, float& dri,
                                               float& drj)
{
    const float u = invr * invr;
    const float xij = Sj * invr, yij = xij * xij;
    const float xji = Si * invr, yji = xji * xji;
    float wij = rcp(1.0f - yij), wji = rcp(1.0f - yji);
    wij *= wij;
    wji *= wji;
    // -r^2 dH/dr = x^3 (P + w) = x (y P + t), r^2 dH/dS = t = y w
    const float tij = yij * wij, tji = yji * wji;
    float aij = xij * fmaf(yij, hct_poly_d(yij), tij);
    float aji = xji * fmaf(yji, hct_poly_d(yji), tji);
    gij2 = tij * u;
    gji2 = tji * u;
    const bool out_ij = (r - Sj >= c) | (c <= rti), out_ji = (r - Si >= c) | (c <= rtj);
    const bool st_ij = !out_ij & (r + Sj > c), st_ji = !out_ji & (r + Si > c);
    const bool f_ij = (r - Sj >= rti) & (yij <= GBMC_HCT_YMAX);
    const bool f_ji = (r - Si >= rtj) & (yji <= GBMC_HCT_YMAX);
    if (!(f_ij & f_ji)) {
        float g[3];
        if (!f_ij) {
            hct_slow32<true>(r, invr, rti, Sj, g);
            aij = -g[0] * r2;
            gij2 = g[2];
            dri = out_ij ? dri : fmaf(bi, g[1], dri);
        }
        if (!f_ji) {
            hct_slow32<true>(r, invr, rtj, Si, g);
            aji = -g[0] * r2;
            gji2 = g[2];
            drj = out_ji ? drj : fmaf(bj, g[1], drj);
        }
    }
    // the part of a straddling ball beyond c: its r and S partials (its rt
    // partial is zero)
    if (st_ij | st_ji) {
        float gc[3];
        if (st_ij) {
            hct_slow32<true>(r, invr, c, Sj, gc);
            aij += gc[0] * r2;
            gij2 -= gc[2];
        }
        if (st_ji) {
            hct_slow32<true>(r, invr, c, Si, gc);
            aji += gc[0] * r2;
            gji2 -= gc[2];
        }
    }
    aij = out_ij ? 0.0f : aij;
    aji = out_ji ? 0.0f : aji;
    gij2 = out_ij ? 0.0f : gij2;
    gji2 = out_ji ? 0.0f : gji2;
    dEdr = -u * fmaf(bi, aij, bj * aji);
}

__device__ __forceinline__ void chain_pair_cut(double r, double r2, double invr, double rti,
                                               double Si, double rtj, double Sj, double bi,
                                               double bj, double c, double& dEdr, double& gij2,
                                               double& gji2, double& dri, double& drj)
{
    const double u = invr * invr;
    const double xij = Sj * invr, yij = xij * xij;
    const double xji = Si * invr, yji = xji * xji;
    double wij = rcp64(1.0 - yij), wji = rcp64(1.0 - yji);
    wij *= wij;
    wji *= wji;
    double aij = xij * yij * (hct_poly64(yij) + wij);
    double aji = xji * yji * (hct_poly64(yji) + wji);
    gij2 = yij * wij * u;
    gji2 = yji * wji * u;
    const bool out_ij = (r - Sj >= c) | (c <= rti), out_ji = (r - Si >= c) | (c <= rtj);
    const bool st_ij = !out_ij & (r + Sj > c), st_ji = !out_ji & (r + Si > c);
    const bool f_ij = (r - Sj >= rti) & (yij <= GBMC_HCT_YMAX64);
    const bool f_ji = (r - Si >= rtj) & (yji <= GBMC_HCT_YMAX64);
    if (!(f_ij & f_ji)) {
        double g0, g1, g2;
        if (!f_ij) {
            hct_general_grad(r, invr, rti, Sj, g0, g1, g2);
            aij = -g0 * r2;
            gij2 = g2;
            dri = out_ij ? dri : fma(bi, g1, dri);
        }
        if (!f_ji) {
            hct_general_grad(r, invr, rtj, Si, g0, g1, g2);
            aji = -g0 * r2;
            gji2 = g2;
            drj = out_ji ? drj : fma(bj, g1, drj);
        }
    }
    if (st_ij | st_ji) {
        double c0, c1, c2;
        if (st_ij) {
            hct_general_grad(r, invr, c, Sj, c0, c1, c2);
            aij += c0 * r2;
            gij2 -= c2;
        }
        if (st_ji) {
            hct_general_grad(r, invr, c, Si, c0, c1, c2);
            aji += c0 * r2;
            gji2 -= c2;
        }
    }
    aij = out_ij ? 0.0 : aij;
    aji = out_ji ? 0.0 : aji;
    gij2 = out_ij ? 0.0 : gij2;
    gji2 = out_ji ? 0.0 : gji2;
    dEdr = -u * fma(bi, aij, bj * aji);
}

// Lower bound of the distance between any atom of one block and any atom of
// another, from their bounding spheres.
__device__ __forceinline__ float block_gap(const Q4<float>& a, const Q4<float>& b)
{
    const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    return sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))) - a.w - b.w;
}

// Whether every pair of an atom of block X with an atom of block Y (X != Y)
// takes the polynomial form of H in both directions, from the staged boxes
// (box[2b]: lowest x, y, z and largest S; box[2b + 1]: highest x, y, z and
// largest rt): the gap g between the boxes bounds every pair distance from
// below, so g >= S_j + rt_i and g >= S_i + rt_j for the blocks' largest S
// and rt give r - S_j >= rt_i and r - S_i >= rt_j, and S^2 <= ymax g^2 gives
// (S / r)^2 <= ymax, for every pair.  The margins (1e-3 A plus 1e-4 relative,
// 0.1 % on ymax) lie far beyond the rounding of the per-pair test and of the
// boxes, so on such a tile that test would pass for every pair: skipping it
// changes no result.
__device__ __forceinline__ bool blocks_separated(const Q4<float>* __restrict__ box, int X, int Y,
                                                 float ymax)
{
    const Q4<float> lx = box[2 * X], hx = box[2 * X + 1];
    const Q4<float> ly = box[2 * Y], hy = box[2 * Y + 1];
    const float gx = fmaxf(0.0f, fmaxf(ly.x - hx.x, lx.x - hy.x));
    const float gy = fmaxf(0.0f, fmaxf(ly.y - hx.y, lx.y - hy.y));
    const float gz = fmaxf(0.0f, fmaxf(ly.z - hx.z, lx.z - hy.z));
    const float g2 = fmaf(gx, gx, fmaf(gy, gy, gz * gz));
    const float need = fmaf(fmaxf(ly.w + hx.w, lx.w + hy.w), 1.0001f, 1e-3f);
    const float sm = fmaxf(lx.w, ly.w);
    return g2 >= need * need && sm * sm <= 0.999f * ymax * g2;
}

// Cutoff work items carry a tile mask: bit k set if j block J0 + k may hold a
// pair within the cutoff (J1 <= J0 + 64).  The first such block at or after
// J, or J1 if none.
__device__ __forceinline__ int next_tile(unsigned long long mask, int J0, int J1, int J)
{
    const int k = J - J0;
    const unsigned long long rest = k < 64 ? mask >> k : 0ull;
    return rest ? J + __builtin_ctzll(rest) : J1;
}

// ---------------------------------------------------------------- helpers

template <typename T>
__device__ __forceinline__ void dummy_pos(int local, T& x, T& y, T& z)
{
    x = T(1.0e6) + T(4096) * T(local);
    y = T(1.0e6);
    z = T(1.0e6);
}

// The waves of a workgroup work on independent items and never wait for each
// other.  Inside one wave, LDS instructions execute in program order, so a
// compiler fence is all that orders a lane's reads after other lanes' writes.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Walks the steps of one tile.  load(s) fetches the j data at LDS slot s;
// pair(d, r, act, acc_j) evaluates the pair of this lane's i row r with that j
// and adds the j-side terms to acc_j (NJ sums); act is false only for the
// lanes that must skip a duplicated pair.  On return acc_j of lane l holds the
// sums of j = 64 J + l.
template <typename T, int NJ, class Load, class Pair>
__device__ __forceinline__ void walk_tile(int lane, bool diagonal, T (&acc_j)[NJ], Load&& load,
                                          Pair&& pair)
{
#pragma unroll
    for (int a = 0; a < NJ; ++a) acc_j[a] = T(0);
    auto step = [&](const auto& d, bool valid) {
        pair(d, 0, valid, acc_j);
#pragma unroll
        for (int a = 0; a < NJ; ++a) acc_j[a] = rot1(acc_j[a]);
    };
    // Two steps per trip with two load buffers, so that the next j is read
    // while the current one is used and no register copies are needed.
    if (!diagonal) {
        auto a = load(lane);
#pragma unroll 1
        for (int k = 0; k < kTile; k += 2) {
            auto b = load(lane + k + 1);
            step(a, true);
            a = load(lane + k + 2);             // slot <= 127: inside the doubled block
            step(b, true);
        }
    } else {
        // pairs (l, l + k) for k = 1..31, and k = 32 for lanes 0..31 only
        auto a = load(lane + 1);
#pragma unroll 1
        for (int k = 1; k < kTile / 2 - 1; k += 2) {
            auto b = load(lane + k + 1);
            step(a, true);
            a = load(lane + k + 2);
            step(b, true);
        }
        auto b = load(lane + kTile / 2);
        step(a, true);
        pair(b, 0, lane < kTile / 2, acc_j);
        // lane l now holds j = l + 32; j = l sits in lane (l - 32) mod 64
#pragma unroll
        for (int a = 0; a < NJ; ++a) acc_j[a] = from_lane(acc_j[a], (lane + kTile / 2) & (kTile - 1));
    }
}

// The same walk for a two-row item (no diagonal): every j serves the pairs of
// both i rows of the lane before the j sums move on.
template <typename T, int NJ, class Load, class Pair>
__device__ __forceinline__ void walk_tile_rows2(int lane, T (&acc_j)[NJ], Load&& load, Pair&& pair)
{
#pragma unroll
    for (int a = 0; a < NJ; ++a) acc_j[a] = T(0);
    auto step = [&](const auto& d) {
        pair(d, 0, true, acc_j);
        pair(d, 1, true, acc_j);
#pragma unroll
        for (int a = 0; a < NJ; ++a) acc_j[a] = rot1(acc_j[a]);
    };
    auto a = load(lane);
#pragma unroll 1
    for (int k = 0; k < kTile; k += 2) {
        auto b = load(lane + k + 1);
        step(a);
        a = load(lane + k + 2);                 // slot <= 127: inside the doubled block
        step(b);
    }
}

// ============================================================ staging
// Packs the caller's SoA inputs into the plan's processing order (a spatial
// order keeps overlapping pairs inside few tiles): P = (x, y, z, q),
// Gx = (rt, S, screen, 0) with rt = rho - offset and S = screen rt.  One wave
// per 64-atom block: lane l stages atom l of the block, and the wave writes
// the block's coordinate box with its largest S and rt (box[2b]: lowest x, y,
// z and S; box[2b + 1]: highest x, y, z and rt), from which the pair passes
// tell the tiles whose pairs all take the polynomial form (blocks_separated).

template <typename T>
__global__ __launch_bounds__(256) void k_stage(const BlockSpan* __restrict__ blocks, int n_blocks,
                                               int n_atoms, const int32_t* __restrict__ perm,
                                               const T* __restrict__ X, const T* __restrict__ Y,
                                               const T* __restrict__ Z, const T* __restrict__ Q,
                                               const T* __restrict__ RHO,
                                               const T* __restrict__ SCR, T offset,
                                               Q4<T>* __restrict__ P, Q4<T>* __restrict__ Gx,
                                               Q4<float>* __restrict__ box, StageClear z)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    // flags and counters of the call start at zero
    if (t < z.n_f0) z.f0[t] = 0;
    if (t < z.n_f1) z.f1[t] = 0;
    for (int i = t; i < z.n_cnt; i += gridDim.x * blockDim.x) z.cnt[i] = 0;
    const int blk = blockIdx.x * 4 + threadIdx.x / kTile, lane = threadIdx.x % kTile;
    if (blk >= n_blocks) return;
    const BlockSpan b = blocks[blk];
    const bool own = lane < b.count;
    const int k = b.start + (own ? lane : b.count - 1);      // count >= 1
    const int c = perm[k];
    Q4<T> p;
    p.x = X[c]; p.y = Y[c]; p.z = Z[c];
    p.w = Q ? Q[c] : T(0);
    Q4<T> g;
    g.x = RHO[c] - offset;
    g.z = SCR[c];
    g.y = g.z * g.x;
    g.w = T(0);
    if (own) {
        // the call's fixed-point accumulators of atom k ([n_acc][N] each) start at zero
        for (int a = 0; a < z.n_acc0; ++a) z.acc0[(size_t)a * n_atoms + k] = 0ull;
        for (int a = 0; a < z.n_acc1; ++a) z.acc1[(size_t)a * n_atoms + k] = 0ull;
        P[k] = p;
        Gx[k] = g;
    }
    // lanes past the end repeat the block's last atom (no effect on the box)
    float lo[4] = {(float)p.x, (float)p.y, (float)p.z, (float)g.y};
    float hi[4] = {lo[0], lo[1], lo[2], (float)g.x};
#pragma unroll
    for (int o = kTile / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], o));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o));
        }
        lo[3] = fmaxf(lo[3], __shfl_xor(lo[3], o));
        hi[3] = fmaxf(hi[3], __shfl_xor(hi[3], o));
    }
    if (lane == 0) {
        box[2 * blk] = Q4<float>{lo[0], lo[1], lo[2], lo[3]};
        box[2 * blk + 1] = Q4<float>{hi[0], hi[1], hi[2], hi[3]};
    }
}

// Bounding sphere of every 64-atom block (centre of the coordinate box,
// radius to the farthest atom, widened by a margin that covers rounding) and
// its largest S, for the cutoff passes: one wave per block.
template <typename T>
__global__ __launch_bounds__(256) void k_block_bounds(const BlockSpan* __restrict__ blocks,
                                                      int n_blocks, const Q4<T>* __restrict__ P,
                                                      const Q4<T>* __restrict__ Gx,
                                                      Q4<float>* __restrict__ bnd,
                                                      float* __restrict__ smax,
                                                      int* __restrict__ ccount)
{
    const int blk = blockIdx.x * 4 + threadIdx.x / kTile, lane = threadIdx.x % kTile;
    // the compaction that follows starts its two lists empty
    if (blockIdx.x == 0 && threadIdx.x < 2) ccount[threadIdx.x] = 0;
    if (blk >= n_blocks) return;
    const BlockSpan b = blocks[blk];
    const int k = b.start + (lane < b.count ? lane : b.count - 1);
    const Q4<T> p = P[k];
    const float x = (float)p.x, y = (float)p.y, z = (float)p.z;
    float lo[3] = {x, y, z}, hi[3] = {x, y, z}, sm = (float)Gx[k].y;
#pragma unroll
    for (int o = kTile / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], o));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o));
        }
        sm = fmaxf(sm, __shfl_xor(sm, o));
    }
    const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
    const float dx = x - cx, dy = y - cy, dz = z - cz;
    float d = sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
#pragma unroll
    for (int o = kTile / 2; o > 0; o >>= 1) d = fmaxf(d, __shfl_xor(d, o));
    if (lane == 0) {
        Q4<float> q;
        q.x = cx; q.y = cy; q.z = cz;
        q.w = d * 1.000001f + 1e-3f;
        bnd[blk] = q;
        smax[blk] = sm;
    }
}

// Compaction of the cutoff passes' work: one wave per chunk (an i block
// against up to 64 j blocks).  Lane k tests j block J0 + k against the
// block bounds; the ballot of the tests is split into items of at most
// kCutTiles tiles.  The 16 waves of a workgroup add their item counts in LDS
// and reserve room in each list with one atomic per workgroup (same-address
// device atomics are the expensive part).  List 0 (descreening and chain
// passes): some ball of one block may reach into the rgbmax sphere of an atom
// of the other; list 1 (energy pass): some pair may lie closer than the pair
// cutoff.  The order of the items varies with the atomics, the results do
// not (integer sums, one rounding unit per tile and per item's i sums).
constexpr int kCutWaves = 16;

__device__ __forceinline__ void write_cut_items(unsigned long long mask, const WorkItem& w,
                                                int lane, int base, CutItem* __restrict__ out,
                                                int cap)
{
    const int n_sub = (__popcll(mask) + kCutTiles - 1) / kCutTiles;
    if (lane < n_sub && base + lane < cap) {
        // the set bits of ranks [lane kCutTiles, (lane + 1) kCutTiles)
        unsigned long long m = mask, sub = 0ull;
        for (int rank = 0; m; ++rank) {
            const unsigned long long low = m & (~m + 1ull);
            m ^= low;
            if (rank / kCutTiles == lane) sub |= low;
        }
        CutItem c;
        c.base = w.base; c.n = w.n; c.I = w.I; c.J0 = w.J0; c.J1 = w.J1; c.blk0 = w.blk0;
        c.mask_lo = (uint32_t)sub;
        c.mask_hi = (uint32_t)(sub >> 32);
        out[base + lane] = c;
    }
}

__global__ __launch_bounds__(kTile * kCutWaves) void k_cut_items(
    const WorkItem* __restrict__ chunks, int n_chunks, const Q4<float>* __restrict__ bnd,
    const float* __restrict__ smax, float cR, float cE, CutItem* __restrict__ out0,
    CutItem* __restrict__ out1, int* __restrict__ ccount, int cap)
{
    __shared__ int cnt[2][kCutWaves];
    __shared__ int base[2];
    const int wave = threadIdx.x / kTile, lane = threadIdx.x % kTile;
    const int ci = blockIdx.x * kCutWaves + wave;
    unsigned long long m0 = 0ull, m1 = 0ull;
    WorkItem w{};
    if (ci < n_chunks) {                         // wave-uniform; every wave reaches the barriers
        w = chunks[ci];
        const Q4<float> bI = bnd[w.blk0 + w.I];
        const float sI = smax[w.blk0 + w.I];
        const int J = w.J0 + lane;
        bool n0 = false, n1 = false;
        if (J < w.J1) {
            const Q4<float> bJ = bnd[w.blk0 + J];
            const float gap = block_gap(bI, bJ);
            n0 = cR > 0.0f && gap - fmaxf(sI, smax[w.blk0 + J]) < cR;
            n1 = cE > 0.0f && gap < cE;
        }
        m0 = __ballot(n0);
        m1 = __ballot(n1);
    }
    if (lane == 0) {
        cnt[0][wave] = (__popcll(m0) + kCutTiles - 1) / kCutTiles;
        cnt[1][wave] = (__popcll(m1) + kCutTiles - 1) / kCutTiles;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        int tot = 0;
        for (int k = 0; k < kCutWaves; ++k) tot += cnt[threadIdx.x][k];
        base[threadIdx.x] = tot > 0 ? atomicAdd(&ccount[threadIdx.x], tot) : 0;
    }
    __syncthreads();
    int off0 = base[0], off1 = base[1];
    for (int k = 0; k < wave; ++k) {
        off0 += cnt[0][k];
        off1 += cnt[1][k];
    }
    write_cut_items(m0, w, lane, off0, out0, cap);
    write_cut_items(m1, w, lane, off1, out1, cap);
}

// ================================================================ pass 1
// I_i = sum_{j != i} H(r_ij; rt_i, S_j) over every unordered pair once.

// One work item: R (1 or 2) consecutive 64-atom i blocks [I, I + R) against
// the j blocks [J0, J1) of one system.  Two-row items hold no diagonal tile
// (J0 >= I + 2): every j read from LDS serves two pairs per lane and the j
// sums move once per two pairs.  Every (i row, j block) tile is rounded into
// fixed point on its own on the i side; the j side of a two-row item rounds
// the sum of its two tiles, the same for every work shape.
template <typename T, int R, bool CUT>
__device__ __forceinline__ void radii_item(const WorkItem& w, int lane, Q4<T>* sj, T* sS,
                                           unsigned long long* sdef, int* slist,
                                           const Q4<T>* __restrict__ P,
                                           const Q4<T>* __restrict__ Gx,
                                           unsigned long long* __restrict__ I_fx,
                                           int* __restrict__ ovf, unsigned long long tmask, T cR,
                                           const Q4<float>* __restrict__ box)
{
    // DEFER (one row, all pairs): overlapping pairs are marked during
    // the walk and evaluated afterwards in packed rounds, as in the chain pass;
    // tiles of separated blocks (blocks_separated) skip the per-pair test and
    // take the short fit of H for y <= YFAR
    constexpr bool DEFER = R == 1 && !CUT;
    constexpr float kYfar = GBMC_HCT_YFAR;    // separated tiles: every pair has y <= this
    T xi[R], yi[R], zi[R], rti[R], Si[R];
    bool vi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = (w.I + r) * kTile + lane;
        vi[r] = i < w.n;
        if (vi[r]) {
            const Q4<T> p = P[w.base + i];
            const Q4<T> gx = Gx[w.base + i];
            xi[r] = p.x; yi[r] = p.y; zi[r] = p.z;
            rti[r] = gx.x;
            Si[r] = gx.y;
        } else {
            dummy_pos(i, xi[r], yi[r], zi[r]);
            rti[r] = T(1);
            Si[r] = T(0);
        }
    }
    // loads of a j block (raw), and the stand-in values of lanes past the end,
    // applied only when the block is written to LDS so the loads stay in flight
    auto fetch = [&](int J, Q4<T>& pj, Q4<T>& gj) {
        const int g = w.base + clamp_atom(J * kTile + lane, w.n);
        pj = P[g];
        gj = Gx[g];
    };
    auto tail = [&](int J, Q4<T>& pj, T& Sj, const Q4<T>& gj) {
        const int j = J * kTile + lane;
        pj.w = gj.x;
        Sj = gj.y;
        if (j >= w.n) {
            dummy_pos(j, pj.x, pj.y, pj.z);
            pj.w = T(1);
            Sj = T(0);
        }
    };
    long long ifix[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ifix[r] = 0;
    bool bad = false;
    Q4<T> pj, gj;
    if constexpr (!CUT) fetch(w.J0, pj, gj);
    // With a cutoff only the tiles of the item's mask are visited.
    int Jnext = w.J1;
    // one tile, then the loads of the next tile; the first tile is peeled so
    // that the loop is entered, as on every later trip, with the previous
    // tile's sums still in flight
    auto tile = [&](int J) {
        int Jn = J + 1;
        if constexpr (CUT) Jnext = Jn = next_tile(tmask, w.J0, w.J1, J + 1);
        const int j = J * kTile + lane;
        const bool vj = j < w.n;
        T Sj;
        tail(J, pj, Sj, gj);
        wave_sync();
        sj[lane] = pj;
        sj[lane + kTile] = pj;
        sS[lane] = Sj;
        sS[lane + kTile] = Sj;
        wave_sync();
        fetch(Jn < w.J1 ? Jn : J, pj, gj);           // the last trip re-reads J
        T ai[R];
#pragma unroll
        for (int r = 0; r < R; ++r) ai[r] = T(0);
        T aj[1];
        struct JD { Q4<T> p; T S; };
        auto load = [&](int s) { return JD{sj[s], sS[s]}; };
        int kstep = J == w.I ? 1 : 0;           // DEFER: walk step of the next pair
        unsigned long long dmask = 0ull;
        auto pair_any = [&](const JD& d, int r, bool act, T (&acc)[1], auto sep_tag) {
            constexpr bool SEP = decltype(sep_tag)::value;
            T hij, hji;
            if constexpr (CUT) {
                radii_pair_cut(xi[r], yi[r], zi[r], d.p.x, d.p.y, d.p.z, rti[r], Si[r], d.p.w, d.S,
                               cR, hij, hji);
            } else if constexpr (DEFER) {
                radii_pair_fast<!SEP>(xi[r], yi[r], zi[r], d.p.x, d.p.y, d.p.z, rti[r], Si[r],
                                      d.p.w, d.S, act && vi[r], 1ull << kstep, hij, hji, dmask);
                ++kstep;
            } else {
                radii_pair(xi[r], yi[r], zi[r], d.p.x, d.p.y, d.p.z, rti[r], Si[r], d.p.w, d.S, hij,
                           hji);
            }
            ai[r] += act ? hij : T(0);
            acc[0] += act ? hji : T(0);
        };
        auto pair = [&](const JD& d, int r, bool act, T (&acc)[1]) {
            pair_any(d, r, act, acc, std::false_type{});
        };
        auto pair_sep = [&](const JD& d, int r, bool act, T (&acc)[1]) {
            pair_any(d, r, act, acc, std::true_type{});
        };
        if constexpr (R == 1) {
            // wave-uniform: the blocks of the tile come from the item
            if (DEFER && J != w.I && blocks_separated(box, w.blk0 + w.I, w.blk0 + J, kYfar))
                walk_tile<T, 1>(lane, false, aj, load, pair_sep);
            else
                walk_tile<T, 1>(lane, J == w.I, aj, load, pair);
        } else {
            walk_tile_rows2<T, 1>(lane, aj, load, pair);
        }
        // DEFER: packed rounds of the marked pairs (see chain_item): j-side
        // terms through LDS integer atomics, i-side terms back to the i lane
        bool deferred = false;
        if constexpr (DEFER) {
            deferred = __builtin_amdgcn_ballot_w64(dmask != 0ull) != 0ull;
            if (deferred) {
                sdef[lane] = 0ull;
                wave_sync();
                for (;;) {
                    const int cnt = __builtin_popcountll(dmask);
                    int incl = cnt;
#pragma unroll
                    for (int dd = 1; dd < kTile; dd <<= 1) {
                        const int o = from_lane_i(incl, (lane - dd) & (kTile - 1));
                        incl += lane >= dd ? o : 0;
                    }
                    const int total = __builtin_amdgcn_readlane(incl, kTile - 1);
                    if (total == 0) break;
                    const int o0 = incl - cnt;
                    const int n = o0 < kTile ? min(cnt, kTile - o0) : 0;
                    for (int t = o0; t < o0 + n; ++t) {
                        const int k = __builtin_ctzll(dmask);
                        dmask &= dmask - 1ull;
                        slist[t] = (lane << 8) | k;
                    }
                    wave_sync();
                    T iv = T(0);
                    if (lane < total) {
                        const int e = slist[lane], il = e >> 8, k = e & 0xff;
                        const int gi = w.base + w.I * kTile + il;
                        const Q4<T> pi = P[gi];
                        const Q4<T> gxi = Gx[gi];       // rt, S
                        const JD d = load(il + k);
                        const T dx = pi.x - d.p.x, dy = pi.y - d.p.y, dz = pi.z - d.p.z;
                        const T r2 = dx * dx + dy * dy + dz * dz;
                        const T invr = rsq(r2);
                        const T rr = r2 * invr;
                        iv = slow_H(rr, invr, gxi.x, d.S);              // H(r; rt_i, S_j)
                        const T hv = slow_H(rr, invr, d.p.w, gxi.y);    // H(r; rt_j, S_i)
                        atomicAdd(&sdef[(il + k) & (kTile - 1)],
                                  (unsigned long long)to_fixed(hv, kScaleI, bad));
                    }
                    for (int u = 0; __builtin_amdgcn_ballot_w64(u < n) != 0ull; ++u) {
                        const T v = from_lane(iv, min(o0 + u, kTile - 1));
                        if (u < n) ai[0] += v;
                    }
                    wave_sync();
                }
            }
        }
        long long hj = to_fixed(aj[0], kScaleI, bad);
        if constexpr (DEFER)
            if (deferred) hj += (long long)sdef[lane];
        fx_add(&I_fx[w.base + clamp_atom(j, w.n)], vj ? hj : 0ll);
#pragma unroll
        for (int r = 0; r < R; ++r) ifix[r] += to_fixed(ai[r], kScaleI, bad);
    };
    if constexpr (CUT) {
        int J = next_tile(tmask, w.J0, w.J1, w.J0);
        if (J >= w.J1) return;                  // nothing within the cutoff: no sums to add
        fetch(J, pj, gj);
        for (; J < w.J1; J = Jnext) tile(J);
    } else {
        tile(w.J0);
        for (int J = w.J0 + 1; J < w.J1; ++J) tile(J);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (vi[r]) fx_add(&I_fx[w.base + (w.I + r) * kTile + lane], ifix[r]);
    if (bad) *ovf = 1;
}

// The compacted items of a cutoff pass, taken in a grid-stride loop (the
// count is known on the device only).
__device__ __forceinline__ WorkItem cut_work_item(const CutItem& c, unsigned long long& mask)
{
    mask = ((unsigned long long)c.mask_hi << 32) | c.mask_lo;
    WorkItem w;
    w.base = c.base; w.n = c.n; w.sys = 0; w.I = c.I; w.J0 = c.J0; w.J1 = c.J1; w.rows = 1;
    w.blk0 = c.blk0;
    return w;
}

template <typename T, int W, bool CUT>
__global__ __launch_bounds__(kTile * W) void k_radii_pairs(
    const WorkItem* __restrict__ items, int n_items, const CutItem* __restrict__ citems,
    const int* __restrict__ n_citems, const Q4<T>* __restrict__ P, const Q4<T>* __restrict__ Gx,
    unsigned long long* __restrict__ I_fx, int* __restrict__ ovf, T cR,
    const Q4<float>* __restrict__ box)
{
    __shared__ Q4<T> sj_w[W][2 * kTile];     // x, y, z, rt
    __shared__ T sS_w[W][2 * kTile];
    // deferred pairs (all-pairs walk only): j-side sums, round list
    constexpr int NL = !CUT ? kTile : 1;
    __shared__ unsigned long long sd_w[W][NL];
    __shared__ int sl_w[W][NL];
    const int wave = threadIdx.x / kTile, lane = threadIdx.x % kTile;
    // the descreening pass runs one-row items only (its two-row form was
    // slower: fewer waves in flight for less saved work)
    if constexpr (CUT) {
        const int n = *n_citems;
        for (int it = __builtin_amdgcn_readfirstlane(blockIdx.x * W + wave); it < n;
             it += gridDim.x * W) {
            unsigned long long m;
            const WorkItem w = cut_work_item(citems[it], m);
            radii_item<T, 1, true>(w, lane, sj_w[wave], sS_w[wave], sd_w[wave], sl_w[wave], P, Gx,
                                   I_fx, ovf, m, cR, box);
        }
    } else {
        // wave-uniform (scalar registers), like everything derived from the item
        const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * W + wave);
        if (item >= n_items) return;
        const WorkItem w = items[item];
        radii_item<T, 1, false>(w, lane, sj_w[wave], sS_w[wave], sd_w[wave], sl_w[wave], P, Gx,
                                I_fx, ovf, 0ull, cR, box);
    }
}

// Per atom: OBC radius from the descreening sum (FP64), and the per-atom state
// of the later passes (FP64 state in caller order, pair-precision copies in
// internal order).
template <typename T>
__device__ __forceinline__ void radii_final_atom(int k, const T* __restrict__ RHO, const GBConst& c,
                                                 const Work<T>& w, T* __restrict__ born_R)
{
    const int g = w.perm[k];
    double rho = (double)RHO[g];
    double rt = rho - c.offset;
    double I = (double)(long long)ld_dev(w.I_fx + k) * (1.0 / kScaleI);
    double psi = rt * I;
    double th = c.alpha * psi - c.beta * psi * psi + c.gamma * psi * psi * psi;
    double t = tanh(th);
    double R = 1.0 / (1.0 / rt - t / rho);
    w.I64[g] = I;
    w.R64[g] = R;
    w.A64[g] = 0.5 / R;
    w.T64[g] = t;
    const double dRdPsi =
        R * R * (1.0 - t * t) * (c.alpha - 2.0 * c.beta * psi + 3.0 * c.gamma * psi * psi) / rho;
    st_dev(w.dRdPsi64 + g, dRdPsi);
    st_dev(w.dRdPsi_p + k, dRdPsi);
    st_dev(w.R_t + k, (T)R);
    st_dev(w.a_t + k, (T)(kAScale / R));
    // FP64 record of the atom for the Monte Carlo kernels (caller order)
    const Q4<T> p = w.P[k];
    Row64 row;
    row.x = (double)p.x; row.y = (double)p.y; row.z = (double)p.z;
    row.R = R; row.A = 0.5 / R;
    row.pad0 = row.pad1 = row.pad2 = 0.0;
    w.rows[g] = row;
    if (born_R) born_R[g] = (T)R;
}

template <typename T>
__global__ void k_radii_finalize(int n_atoms, const T* __restrict__ RHO, GBConst c, Work<T> w,
                                 T* __restrict__ born_R)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_atoms) return;
    radii_final_atom<T>(k, RHO, c, w, born_R);
}

// ================================================================ pass 2
// Coulomb + GB energy, explicit pair forces, G = dE/dR, phi = dE/dq.

// One work item of R (1 or 2) i blocks; see radii_item.
template <typename T, bool GRAD, int R, bool SALT, bool CUT, bool ONE>
__device__ __forceinline__ void energy_item(const WorkItem& w, int lane, Q4<T>* sj, T* sR, T* sA,
                                            const Q4<T>* __restrict__ P, const T* __restrict__ Rt,
                                            const T* __restrict__ At, T kC, T kT,
                                            const SaltK<T>& sk, const CutK<T>& ck,
                                            const Work<T>& wk, unsigned long long tmask)
{
    constexpr int NJ = GRAD ? 5 : 1;
    // Without salt the pair terms take the charges scaled by sqrt(kC), so that
    // qq = kC q_i q_j carries the Coulomb constant and tau = kT / kC the GB
    // factor; the phi and G sums are rescaled when they are rounded (sPhi,
    // sG), which saves four multiplications per pair.  With salt the factors
    // vary per pair and the charges stay as given.
    const T sq = SALT ? T(1) : T(sqrt(kC));
    const T tau = SALT || kC == T(0) ? T(0) : kT / kC;
    const T qtau = T(-0.25) * tau;
    const T sPhi = sq, sG = SALT ? T(1) : T(0.5) * tau;
    T xi[R], yi[R], zi[R], qi[R], Ri[R], ai[R];
    bool vi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = (w.I + r) * kTile + lane;
        vi[r] = i < w.n;
        if (vi[r]) {
            const int g = w.base + i;
            const Q4<T> p = P[g];
            xi[r] = p.x; yi[r] = p.y; zi[r] = p.z; qi[r] = p.w * sq;
            Ri[r] = ld_dev(Rt + g); ai[r] = ld_dev(At + g);
        } else {
            dummy_pos(i, xi[r], yi[r], zi[r]);
            qi[r] = T(0); Ri[r] = T(1); ai[r] = T(kAScale);
        }
    }
    // raw loads of a j block; stand-ins for lanes past the end are applied
    // when the block is written to LDS
    auto fetch = [&](int J, Q4<T>& pj, T& Rj, T& Aj) {
        const int g = w.base + clamp_atom(J * kTile + lane, w.n);
        pj = P[g];
        Rj = ld_dev(Rt + g); Aj = ld_dev(At + g);
    };
    auto tail = [&](int J, Q4<T>& pj, T& Rj, T& Aj) {
        const int j = J * kTile + lane;
        if (j >= w.n) {
            dummy_pos(j, pj.x, pj.y, pj.z);
            pj.w = T(0);
            Rj = T(1); Aj = T(kAScale);
        }
    };
    long long fix[R][5], efix[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int a = 0; a < 5; ++a) fix[r][a] = 0;
        efix[r][0] = efix[r][1] = 0;
    }
    bool bad = false;
    Q4<T> pj;
    T Rj, Aj;
    if constexpr (!CUT) fetch(w.J0, pj, Rj, Aj);
    // With a cutoff only the tiles of the item's mask are visited.
    int Jnext = w.J1;
    // one tile, then the loads of the next tile; the first tile is peeled so
    // that the loop is entered, as on every later trip, with the previous
    // tile's sums still in flight
    // FIRST (the peeled first tile of a full item): the i-side sums are set,
    // not added to, so no zeroed accumulators stay live through the walk
    auto tile = [&](int J, auto first_tag) {
        constexpr bool FIRST = decltype(first_tag)::value;
        int Jn = J + 1;
        if constexpr (CUT) Jnext = Jn = next_tile(tmask, w.J0, w.J1, J + 1);
        const int j = J * kTile + lane;
        const bool vj = j < w.n;
        tail(J, pj, Rj, Aj);
        Q4<T> ps = pj;
        ps.w *= sq;
        wave_sync();
        sj[lane] = ps;
        sR[lane] = Rj;
        sA[lane] = Aj;
        wave_sync();
        fetch(Jn < w.J1 ? Jn : J, pj, Rj, Aj);
        T fxi[R], fyi[R], fzi[R], Gi[R], phii[R], eC[R], eG[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            fxi[r] = fyi[r] = fzi[r] = Gi[r] = phii[r] = eC[r] = eG[r] = T(0);
        T aj[NJ];
        struct JD { Q4<T> p; T Rv, Av; };
        // one copy of the block, read at slot (lane + step) mod 64 (measured
        // faster here than the doubled copy the other passes read without a wrap)
        auto load = [&](int s) {
            const int m = s & (kTile - 1);
            return JD{sj[m], sR[m], sA[m]};
        };
        auto pair = [&](const JD& d, int r, bool act, T (&acc)[NJ]) {
            const Q4<T>& p = d.p;
            const T rj = d.Rv;
            T dx = xi[r] - p.x, dy = yi[r] - p.y, dz = zi[r] - p.z;
            T r2 = dx * dx + dy * dy + dz * dz;
            if constexpr (CUT) act = act && r2 < ck.cE2;     // pairs beyond the cutoff drop out
            T invr = rsq(r2);
            T t = r2 * (ai[r] * d.Av);            // r^2 log2(e) / (4 R_i R_j)
            T ex = exp2neg(t);                   // exp(-D)
            T f2 = Ri[r] * rj * ex + r2;
            T invf = rsq(f2);
            T qq = act ? qi[r] * p.w : T(0);
            eC[r] += qq * invr;
            // GB factor of the pair: with salt kd = k (1/eps_in -
            // exp(-kappa f)/eps_out) and the slope factor ks = kd - k kappa f
            // exp(-kappa f)/eps_out (d/df (kd/f) = -ks/f^2); without salt both
            // are kT = k (1/eps_in - 1/eps_out) = tau kC, carried by the scaled
            // charges and tau
            [[maybe_unused]] T kd = kT, ks = kT;
            if constexpr (SALT) {
                const T f = f2 * invf;
                const T es = sk.kO * exp2neg(sk.kap2 * f);
                kd = kC - es;
                ks = kd - es * sk.kap * f;
                eG[r] += qq * kd * invf;
            } else {
                eG[r] += qq * invf;
            }
            if constexpr (GRAD) {
                T qj = act ? p.w : T(0);
                T qi_ = act ? qi[r] : T(0);
                T invf3 = invf * invf * invf;
                T invr3 = invr * invr * invr;
                T wgt, fr, cg;
                if constexpr (SALT) {
                    wgt = kC * invr - kd * invf;
                    fr = qq * (ks * invf3 * (T(1) - T(0.25) * ex) - kC * invr3);   // (dE/dr)/r
                    cg = T(0.5) * ks * qq * invf3 * ex * (T(1) + t * T(kLn2));
                } else {
                    // scaled charges: phi weight over sqrt(kC), G term over tau / 2
                    wgt = invr - tau * invf;
                    fr = qq * ((ex * qtau + tau) * invf3 - invr3);
                    cg = qq * invf3 * ex * (T(1) + t * T(kLn2));
                }
                phii[r] += wgt * qj;
                T fx = fr * dx, fy = fr * dy, fz = fr * dz;
                fxi[r] -= fx; fyi[r] -= fy; fzi[r] -= fz;
                Gi[r] += cg * rj;
                acc[0] += fx;
                acc[1] += fy;
                acc[2] += fz;
                acc[3] += cg * Ri[r];
                acc[4] += wgt * qi_;
            }
        };
        if constexpr (R == 1)
            walk_tile<T, NJ>(lane, J == w.I, aj, load, pair);
        else
            walk_tile_rows2<T, NJ>(lane, aj, load, pair);
        if (R == 1 && J == w.I) {
            // self terms (f_ii = R_i): -(kd/2) q_i^2 / R_i in E_GB, -kd q_i / R_i
            // in phi, (ks/2) q_i^2 / R_i^2 in G (without salt in the scaled
            // form of the walk's sums)
            T invR = rcp(Ri[0]);
            [[maybe_unused]] T kd = kT, ks = kT;
            if constexpr (SALT) {
                const T es = sk.kO * exp2neg(sk.kap2 * Ri[0]);
                kd = kC - es;
                ks = kd - es * sk.kap * Ri[0];
                eG[0] += T(0.5) * qi[0] * qi[0] * kd * invR;
                if constexpr (GRAD) {
                    phii[0] -= kd * qi[0] * invR;
                    Gi[0] += T(0.5) * ks * qi[0] * qi[0] * invR * invR;
                }
            } else {
                eG[0] += T(0.5) * qi[0] * qi[0] * invR;
                if constexpr (GRAD) {
                    phii[0] -= tau * qi[0] * invR;
                    Gi[0] += qi[0] * qi[0] * invR * invR;
                }
            }
        }
        if constexpr (GRAD) {
            const int g = w.base + clamp_atom(j, w.n);
            long long v[5];
            aj[3] *= sG;
            aj[4] *= sPhi;
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                v[a] = to_fixed(aj[a], kScaleF, bad);
                v[a] = vj ? v[a] : 0ll;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) fx_add(&wk.F_fx[a * wk.n_atoms + g], v[a]);
            fx_add(&wk.G_fx[g], v[3]);
            fx_add(&wk.phi_fx[g], v[4]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const long long f[5] = {to_fixed(fxi[r], kScaleF, bad), to_fixed(fyi[r], kScaleF, bad),
                                        to_fixed(fzi[r], kScaleF, bad),
                                        to_fixed(T(Gi[r] * sG), kScaleF, bad),
                                        to_fixed(T(phii[r] * sPhi), kScaleF, bad)};
#pragma unroll
                for (int a = 0; a < 5; ++a) fix[r][a] = FIRST ? f[a] : fix[r][a] + f[a];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // Coulomb: kC is in qq without salt; GB: -tau (scaled charges) or -1
            // (salt: the factor is in every term)
            const long long e0 = to_fixed(T((SALT ? kC : T(1)) * eC[r]), kScaleE, bad);
            const long long e1 = to_fixed(T(-(SALT ? T(1) : tau) * eG[r]), kScaleE, bad);
            efix[r][0] = FIRST ? e0 : efix[r][0] + e0;
            efix[r][1] = FIRST ? e1 : efix[r][1] + e1;
        }
    };
    if constexpr (CUT) {
        int J = next_tile(tmask, w.J0, w.J1, w.J0);
        if (J >= w.J1) return;                  // nothing within the cutoff: no sums to add
        fetch(J, pj, Rj, Aj);
        for (; J < w.J1; J = Jnext) tile(J, std::false_type{});
    } else {
        tile(w.J0, std::true_type{});
        // ONE: every item of the launch is a single tile (one j block); the
        // prefetch and the cross-tile sums then drop out, and the kernel
        // needs fewer registers
        if constexpr (!ONE)
            for (int J = w.J0 + 1; J < w.J1; ++J) tile(J, std::false_type{});
    }
    if (bad) *wk.ovf = 1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!vi[r]) continue;
        const int g = w.base + (w.I + r) * kTile + lane;
        if constexpr (GRAD) {
#pragma unroll
            for (int a = 0; a < 3; ++a) fx_add(&wk.F_fx[a * wk.n_atoms + g], fix[r][a]);
            fx_add(&wk.G_fx[g], fix[r][3]);
            fx_add(&wk.phi_fx[g], fix[r][4]);
        }
        // energies: each atom's share, summed per system by k_energy_finalize
        // (exact integers, so the split into atoms does not change the totals)
        fx_add(&wk.EA_fx[g], efix[r][0]);
        fx_add(&wk.EA_fx[wk.n_atoms + g], efix[r][1]);
    }
}

template <typename T, bool GRAD, int W, bool SALT, bool CUT, bool ONE>
__global__ __launch_bounds__(kTile * W) void k_energy_pairs(
    const WorkItem* __restrict__ items, int n_items, const Q4<T>* __restrict__ P,
    const T* __restrict__ Rt, const T* __restrict__ At, T kC, T kT, SaltK<T> sk, CutK<T> ck,
    Work<T> wk)
{
    __shared__ Q4<T> sj_w[W][kTile];     // x, y, z, q
    __shared__ T sR_w[W][kTile];
    __shared__ T sA_w[W][kTile];
    const int wave = threadIdx.x / kTile, lane = threadIdx.x % kTile;
    if constexpr (CUT) {
        // compacted one-row items of the pair cutoff
        const int n = wk.ccount[1];
        for (int it = __builtin_amdgcn_readfirstlane(blockIdx.x * W + wave); it < n;
             it += gridDim.x * W) {
            unsigned long long m;
            const WorkItem w = cut_work_item(wk.citems[1][it], m);
            energy_item<T, GRAD, 1, SALT, true, false>(w, lane, sj_w[wave], sR_w[wave], sA_w[wave], P, Rt,
                                                At, kC, kT, sk, ck, wk, m);
        }
    } else {
        // wave-uniform (scalar registers), like everything derived from the item
        const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * W + wave);
        if (item >= n_items) return;
        const WorkItem w = items[item];
        // two-row items exist in the energy pass of FP32 plans only
        if (sizeof(T) == 4 && w.rows == 2)
            energy_item<T, GRAD, sizeof(T) == 4 ? 2 : 1, SALT, false, ONE>(w, lane, sj_w[wave],
                                                                      sR_w[wave], sA_w[wave], P,
                                                                      Rt, At, kC, kT, sk, ck, wk,
                                                                      0ull);
        else
            energy_item<T, GRAD, 1, SALT, false, ONE>(w, lane, sj_w[wave], sR_w[wave], sA_w[wave], P, Rt,
                                                 At, kC, kT, sk, ck, wk, 0ull);
    }
}

// After pass 2, one launch: blocks [0, n_sum) sum the atoms' fixed-point
// energy shares of one system each (E_C, E_GB; integer sums, so the result
// does not depend on the order), the following blocks finalize one atom per
// thread: B = G dR/dPsi for the chain pass and the dE/dq output.
template <typename T>
__global__ __launch_bounds__(256) void k_energy_finalize(int n_atoms, int n_sum, Work<T> w,
                                                         double* __restrict__ e_coul,
                                                         double* __restrict__ e_gb,
                                                         T* __restrict__ dEdq, bool grad)
{
    const int t = threadIdx.x;
    if ((int)blockIdx.x < n_sum) {
        __shared__ long long part[2][4];
        const int b = blockIdx.x, lane = t % kTile, wave = t / kTile;
        const unsigned long long* EA = w.EA_fx;
        long long s0 = 0, s1 = 0;
        for (int g = w.atom_offset[b] + t; g < w.atom_offset[b + 1]; g += 256) {
            s0 += (long long)EA[g];
            s1 += (long long)EA[w.n_atoms + g];
        }
#pragma unroll
        for (int o = kTile / 2; o > 0; o >>= 1) {
            s0 += __shfl_xor(s0, o);
            s1 += __shfl_xor(s1, o);
        }
        if (lane == 0) { part[0][wave] = s0; part[1][wave] = s1; }
        __syncthreads();
        if (t == 0) {
            long long c = part[0][0] + part[0][1] + part[0][2] + part[0][3];
            long long gb = part[1][0] + part[1][1] + part[1][2] + part[1][3];
            if (e_coul) e_coul[b] = (double)c * (1.0 / kScaleE);
            if (e_gb) e_gb[b] = (double)gb * (1.0 / kScaleE);
        }
        return;
    }
    const int k = ((int)blockIdx.x - n_sum) * 256 + t;
    if (!grad || k >= n_atoms) return;
    if (dEdq) dEdq[w.perm[k]] = (T)((double)(long long)w.phi_fx[k] * (1.0 / kScaleF));
}

// ================================================================ pass 3
// Born-radius chain: force through Psi and the pair part of dE/drho.

// One work item of R (1 or 2) i blocks; see radii_item.
// B (rho - offset) of one atom in the pair precision, formed from its G sum
// (fixed point, final once the energy pass is) and dR/dPsi: B = G dR/dPsi in
// FP64, then one rounding to the pair precision (the output kernel forms the
// same FP64 B), so no finalize launch is needed between the energy and chain
// passes.
template <typename T>
__device__ __forceinline__ T brt_from(unsigned long long gfx, double dRdPsi, T rt)
{
    const double G = (double)(long long)gfx * (1.0 / kScaleF);
    const double B = G * dRdPsi;
    return (T)(B * (double)rt);
}

template <typename T, int R, bool CUT, bool ONE>
__device__ __forceinline__ void chain_item(const WorkItem& w, int lane, Q4<T>* sj, Q4<T>* sb,
                                           unsigned long long* sdef, int* slist,
                                           const Q4<T>* __restrict__ P,
                                           const Q4<T>* __restrict__ Gx,
                                           const Work<T>& wk, T cR,
                                           unsigned long long tmask)
{
    // DEFER (all pairs): the walk evaluates the polynomial form only and
    // marks the pairs that need the closed form (overlapping spheres) in a
    // per-lane, per-row mask of walk steps; after the walk the marked pairs
    // are evaluated packed, one per lane per round, instead of with most of
    // the wave masked off in the step that met them.  Their j-side terms go to
    // the j atoms through LDS int64 fixed-point atomics (exact, so the result
    // does not depend on the order of the rounds).
    constexpr bool DEFER = !CUT;
    constexpr float kYfar = GBMC_HCT_YFAR;    // separated tiles: every pair has y <= this
    T xi[R], yi[R], zi[R], rti[R], Si[R], Bi[R], si[R];
    bool vi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = (w.I + r) * kTile + lane;
        vi[r] = i < w.n;
        if (vi[r]) {
            const int g = w.base + i;
            const Q4<T> p = P[g];
            const Q4<T> gx = Gx[g];
            xi[r] = p.x; yi[r] = p.y; zi[r] = p.z;
            rti[r] = gx.x;
            Si[r] = gx.y;
            si[r] = gx.z;
            Bi[r] = brt_from<T>(ld_dev(wk.G_fx + g), ld_dev(wk.dRdPsi_p + g), gx.x);
        } else {
            dummy_pos(i, xi[r], yi[r], zi[r]);
            rti[r] = T(1); si[r] = T(0); Si[r] = T(0); Bi[r] = T(0);
        }
    }
    // raw loads of a j block; stand-ins for lanes past the end are applied
    // when the block is written to LDS
    // raw loads of a j block (G sum and dR/dPsi for its B rt, formed when the
    // block is written to LDS so that the loads stay in flight)
    auto fetch = [&](int J, Q4<T>& pj, Q4<T>& gj, unsigned long long& gfj, double& drj) {
        const int g = w.base + clamp_atom(J * kTile + lane, w.n);
        pj = P[g];
        gj = Gx[g];
        gfj = ld_dev(wk.G_fx + g);
        drj = ld_dev(wk.dRdPsi_p + g);
    };
    auto tail = [&](int J, Q4<T>& pj, Q4<T>& bj, const Q4<T>& gj, unsigned long long gfj,
                    double drj) {
        const int j = J * kTile + lane;
        pj.w = gj.x;
        bj.x = gj.y;
        bj.y = brt_from<T>(gfj, drj, gj.x);
        bj.z = gj.z;
        bj.w = T(0);
        if (j >= w.n) {
            dummy_pos(j, pj.x, pj.y, pj.z);
            pj.w = T(1);
            bj.x = bj.y = bj.z = T(0);
        }
    };
    long long fix[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) fix[r][0] = fix[r][1] = fix[r][2] = fix[r][3] = 0;
    bool bad = false;
    Q4<T> pj, gj, bj;
    unsigned long long gfj;
    double drj;
    if constexpr (!CUT) fetch(w.J0, pj, gj, gfj, drj);
    // With a cutoff only the tiles of the item's mask are visited.
    int Jnext = w.J1;
    // one tile, then the loads of the next tile; the first tile is peeled so
    // that the loop is entered, as on every later trip, with the previous
    // tile's sums still in flight
    // FIRST: as in the energy pass, the first tile sets the i-side sums
    auto tile = [&](int J, auto first_tag) {
        constexpr bool FIRST = decltype(first_tag)::value;
        int Jn = J + 1;
        if constexpr (CUT) Jnext = Jn = next_tile(tmask, w.J0, w.J1, J + 1);
        const int j = J * kTile + lane;
        const bool vj = j < w.n;
        tail(J, pj, bj, gj, gfj, drj);
        wave_sync();
        sj[lane] = pj; sj[lane + kTile] = pj;
        sb[lane] = bj; sb[lane + kTile] = bj;
        wave_sync();
        fetch(Jn < w.J1 ? Jn : J, pj, gj, gfj, drj);
        T fxi[R], fyi[R], fzi[R], dri[R];
#pragma unroll
        for (int r = 0; r < R; ++r) fxi[r] = fyi[r] = fzi[r] = dri[r] = T(0);
        T aj[4];
        struct JD { Q4<T> p, b; };
        auto load = [&](int s) { return JD{sj[s], sb[s]}; };
        // DEFER: walk step of the next pair call (the walk visits slot lane + k
        // at step k: k = 0..63 off the diagonal, 1..32 on it) and the marks
        int kstep = J == w.I ? 1 : 0;
        unsigned long long dmask[R];
#pragma unroll
        for (int r = 0; r < R; ++r) dmask[r] = 0ull;
        auto pair_any = [&](const JD& d, int r, bool act, T (&acc)[4], auto sep_tag) {
            constexpr bool SEP = decltype(sep_tag)::value;
            const Q4<T>& p = d.p;
            const Q4<T>& b = d.b;
            T dx = xi[r] - p.x, dy = yi[r] - p.y, dz = zi[r] - p.z;
            T r2 = dx * dx + dy * dy + dz * dz;
            T invr = rsq(r2);
            T rr = r2 * invr;
            const T bj_ = act ? b.y : T(0);
            const T bi_ = act ? Bi[r] : T(0);
            T dEdr, gij2, gji2;
            if constexpr (CUT) {
                chain_pair_cut(rr, r2, invr, rti[r], Si[r], p.w, b.x, bi_, bj_, cR, dEdr, gij2, gji2,
                               dri[r], acc[3]);
            } else if constexpr (DEFER) {
                // only pairs of a real i atom are marked (padding lanes sit far
                // apart, so none of theirs needs the closed form anyway); the
                // packed rounds read the i atom back from global memory
                chain_pair_fast<!SEP>(rr, invr, rti[r], Si[r], p.w, b.x, bi_, bj_, act && vi[r],
                                      1ull << kstep, dEdr, gij2, gji2, dmask[r]);
                if (r == R - 1) ++kstep;            // a step serves every row of the item
            } else {
                chain_pair(rr, r2, invr, rti[r], Si[r], p.w, b.x, bi_, bj_, dEdr, gij2, gji2,
                           dri[r], acc[3]);
            }
            T fr = dEdr * invr;
            T fx = fr * dx, fy = fr * dy, fz = fr * dz;
            fxi[r] -= fx; fyi[r] -= fy; fzi[r] -= fz;
            dri[r] += si[r] * bj_ * gji2;
            acc[0] += fx;
            acc[1] += fy;
            acc[2] += fz;
            acc[3] += b.z * bi_ * gij2;
        };
        auto pair = [&](const JD& d, int r, bool act, T (&acc)[4]) {
            pair_any(d, r, act, acc, std::false_type{});
        };
        auto pair_sep = [&](const JD& d, int r, bool act, T (&acc)[4]) {
            pair_any(d, r, act, acc, std::true_type{});
        };
        if constexpr (R == 1) {
            // separated blocks (wave-uniform): no pair needs the closed form
            if (DEFER && J != w.I && blocks_separated(wk.box, w.blk0 + w.I, w.blk0 + J, kYfar))
                walk_tile<T, 4>(lane, false, aj, load, pair_sep);
            else
                walk_tile<T, 4>(lane, J == w.I, aj, load, pair);
        } else {
            // two rows (never a diagonal tile): separated if both rows' tiles are
            if (DEFER && blocks_separated(wk.box, w.blk0 + w.I, w.blk0 + J, kYfar) &&
                blocks_separated(wk.box, w.blk0 + w.I + 1, w.blk0 + J, kYfar))
                walk_tile_rows2<T, 4>(lane, aj, load, pair_sep);
            else
                walk_tile_rows2<T, 4>(lane, aj, load, pair);
        }
        // DEFER: the marked pairs, packed into rounds of up to 64 (the marks of
        // all lanes listed in lane order, lane t of a round taking list entry
        // t).  The j-side terms are rounded to fixed point per pair and added
        // with LDS integer atomics (sdef[a * 64 + j lane]: exact, so the order
        // of a round's lanes does not matter); the i-side terms go back to the
        // i atom's lane, which owns a contiguous run of the round's entries
        // (its first row's marks, then its second row's), and join its FP32
        // sums in list order.
        bool deferred = false;
        if constexpr (DEFER) {
            unsigned long long any = 0ull;
#pragma unroll
            for (int r = 0; r < R; ++r) any |= dmask[r];
            deferred = __builtin_amdgcn_ballot_w64(any != 0ull) != 0ull;
            if (deferred) {
#pragma unroll
                for (int a = 0; a < 4; ++a) sdef[a * kTile + lane] = 0ull;
                wave_sync();
                for (;;) {
                    const int cnt0 = __builtin_popcountll(dmask[0]);
                    const int cnt = R == 1 ? cnt0 : cnt0 + __builtin_popcountll(dmask[R - 1]);
                    int incl = cnt;                     // inclusive scan over the lanes
#pragma unroll
                    for (int d = 1; d < kTile; d <<= 1) {
                        const int o = from_lane_i(incl, (lane - d) & (kTile - 1));
                        incl += lane >= d ? o : 0;
                    }
                    const int total = __builtin_amdgcn_readlane(incl, kTile - 1);
                    if (total == 0) break;
                    // this lane's entries of the round: list slots [o0, o0 + n)
                    const int o0 = incl - cnt;
                    const int n = o0 < kTile ? min(cnt, kTile - o0) : 0;
                    const int n0 = min(n, cnt0);        // entries [0, n0) of the run: first row
                    for (int t = o0; t < o0 + n; ++t) {
                        int k, ir;
                        if (R == 1 || dmask[0] != 0ull) {
                            k = __builtin_ctzll(dmask[0]);
                            dmask[0] &= dmask[0] - 1ull;
                            ir = 0;
                        } else {
                            k = __builtin_ctzll(dmask[R - 1]);
                            dmask[R - 1] &= dmask[R - 1] - 1ull;
                            ir = 1;
                        }
                        slist[t] = (lane << 8) | (ir << 7) | k;
                    }
                    wave_sync();
                    T iv[4] = {T(0), T(0), T(0), T(0)};
                    if (lane < total) {
                        const int e = slist[lane], il = e >> 8, k = e & 0x7f;
                        const int gi = w.base + (w.I + ((e >> 7) & 1)) * kTile + il;
                        const Q4<T> pi = P[gi];
                        const Q4<T> gxi = Gx[gi];       // rt, S, screen
                        const T bi_ = brt_from<T>(ld_dev(wk.G_fx + gi),
                                                  ld_dev(wk.dRdPsi_p + gi), gxi.x);
                        const JD d = load(il + k);
                        const Q4<T>& p = d.p;
                        const Q4<T>& b = d.b;
                        const T dx = pi.x - p.x, dy = pi.y - p.y, dz = pi.z - p.z;
                        const T r2 = dx * dx + dy * dy + dz * dz;
                        const T invr = rsq(r2);
                        const T rr = r2 * invr;
                        T ga[3], gb[3];
                        slow_grad(rr, invr, gxi.x, b.x, ga);            // H(r; rt_i, S_j)
                        slow_grad(rr, invr, p.w, gxi.y, gb);            // H(r; rt_j, S_i)
                        const T bj_ = b.y;
                        // dE/dr = bi dH_ij/dr + bj dH_ji/dr
                        const T fr = T(fma(bi_, ga[0], bj_ * gb[0])) * invr;
                        const T fx = fr * dx, fy = fr * dy, fz = fr * dz;
                        iv[0] = -fx; iv[1] = -fy; iv[2] = -fz;
                        iv[3] = T(fma(bi_, ga[1], gxi.z * bj_ * gb[2]));
                        const T jv[4] = {fx, fy, fz, T(fma(b.z * bi_, ga[2], bj_ * gb[1]))};
                        const int jl = (il + k) & (kTile - 1);
#pragma unroll
                        for (int a = 0; a < 4; ++a)
                            atomicAdd(&sdef[a * kTile + jl],
                                      (unsigned long long)to_fixed(jv[a], kScaleF, bad));
                    }
                    // i side: every lane reads its run (all lanes take part in
                    // each read, the sums only for u < n)
                    for (int u = 0; __builtin_amdgcn_ballot_w64(u < n) != 0ull; ++u) {
                        const int src = min(o0 + u, kTile - 1);
                        const T v0 = from_lane(iv[0], src), v1 = from_lane(iv[1], src);
                        const T v2 = from_lane(iv[2], src), v3 = from_lane(iv[3], src);
                        if (u < n) {
                            if (R == 1 || u < n0) {
                                fxi[0] += v0; fyi[0] += v1; fzi[0] += v2; dri[0] += v3;
                            } else {
                                fxi[R - 1] += v0; fyi[R - 1] += v1; fzi[R - 1] += v2;
                                dri[R - 1] += v3;
                            }
                        }
                    }
                    wave_sync();
                }
            }
        }
        {
            const int g = w.base + clamp_atom(j, w.n);
            long long v[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                v[a] = to_fixed(aj[a], kScaleF, bad);
                if constexpr (DEFER)
                    if (deferred) v[a] += (long long)sdef[a * kTile + lane];
                v[a] = vj ? v[a] : 0ll;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) fx_add(&wk.F_fx[a * wk.n_atoms + g], v[a]);
            fx_add(&wk.drho_fx[g], v[3]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const long long f[4] = {to_fixed(fxi[r], kScaleF, bad), to_fixed(fyi[r], kScaleF, bad),
                                    to_fixed(fzi[r], kScaleF, bad), to_fixed(dri[r], kScaleF, bad)};
#pragma unroll
            for (int a = 0; a < 4; ++a) fix[r][a] = FIRST ? f[a] : fix[r][a] + f[a];
        }
    };
    if constexpr (CUT) {
        int J = next_tile(tmask, w.J0, w.J1, w.J0);
        if (J >= w.J1) return;                  // nothing within the cutoff: no sums to add
        fetch(J, pj, gj, gfj, drj);
        for (; J < w.J1; J = Jnext) tile(J, std::false_type{});
    } else {
        tile(w.J0, std::true_type{});
        if constexpr (!ONE)                     // ONE: single-tile items, as in the energy pass
            for (int J = w.J0 + 1; J < w.J1; ++J) tile(J, std::false_type{});
    }
    if (bad) *wk.ovf = 1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!vi[r]) continue;
        const int g = w.base + (w.I + r) * kTile + lane;
#pragma unroll
        for (int a = 0; a < 3; ++a) fx_add(&wk.F_fx[a * wk.n_atoms + g], fix[r][a]);
        fx_add(&wk.drho_fx[g], fix[r][3]);
    }
}

template <typename T, int W, bool CUT, bool ONE>
__global__ __launch_bounds__(kTile * W) void k_chain_pairs(
    const WorkItem* __restrict__ items, int n_items, const Q4<T>* __restrict__ P,
    const Q4<T>* __restrict__ Gx, Work<T> wk, T cR)
{
    __shared__ Q4<T> sj_w[W][2 * kTile];     // x, y, z, rt
    __shared__ Q4<T> sb_w[W][2 * kTile];     // S, B rt, screen, -
    // deferred pairs (all-pairs walk only): j-side sums, round list
    constexpr int ND = !CUT ? 4 * kTile : 1;
    constexpr int NL = !CUT ? kTile : 1;
    __shared__ unsigned long long sd_w[W][ND];
    __shared__ int sl_w[W][NL];
    const int wave = threadIdx.x / kTile, lane = threadIdx.x % kTile;
    if constexpr (CUT) {
        const int n = wk.ccount[0];
        for (int it = __builtin_amdgcn_readfirstlane(blockIdx.x * W + wave); it < n;
             it += gridDim.x * W) {
            unsigned long long m;
            const WorkItem w = cut_work_item(wk.citems[0][it], m);
            chain_item<T, 1, true, false>(w, lane, sj_w[wave], sb_w[wave], sd_w[wave], sl_w[wave], P,
                                          Gx, wk, cR, m);
        }
    } else {
        // wave-uniform (scalar registers), like everything derived from the item
        const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * W + wave);
        if (item >= n_items) return;
        const WorkItem w = items[item];
        // two-row items exist in the chain and energy passes of FP32 plans only
        if (sizeof(T) == 4 && w.rows == 2)
            chain_item<T, sizeof(T) == 4 ? 2 : 1, false, ONE>(w, lane, sj_w[wave], sb_w[wave],
                                                            sd_w[wave], sl_w[wave], P, Gx, wk,
                                                            cR, 0ull);
        else
            chain_item<T, 1, false, ONE>(w, lane, sj_w[wave], sb_w[wave], sd_w[wave], sl_w[wave], P,
                                         Gx, wk, cR, 0ull);
    }
}


// ===================================================== one queued launch
// The pair passes of one call (descreening, energy / explicit forces, Born
// chain; all pairs) run as one launch.  Its work items form one sequence, in
// pass order (within a pass as the plan lists them).  Every workgroup takes
// the next ticket from a device counter when it starts and its W waves run the
// W consecutive items of that ticket, so the items start in sequence order.
// An item of a later pass first waits until every 64-atom block it touches is
// final in the preceding pass: every item counts itself done on each of its
// blocks (int counters), and the wave whose count completes a block marks it
// ready (count + 1), after the descreening pass once it has finalized the
// block (the OBC radius and its derivatives; after the energy pass the block's
// G sums are final, from which the chain items form the chain weights).
// Every wait ends: an item waits only for items earlier in the sequence, which
// were taken by workgroups that started before it (or by its own workgroup)
// and so are running or done.  Each wait is bounded all the same
// (PQueue::spin_limit polls): a wave that gives up sets the launch's error
// word and skips its item, every later wait then gives up at once, so the
// launch drains, and the host reads the error (gbmc_check_overflow).
// Counters, fixed-point sums and block finals move between the waves through
// device-scope atomics, loads and stores (coherent across the XCDs' L2
// caches).  (A grid of resident workgroups that loop over the sequence was
// measured to need 30-50 % more registers per wave, hence fewer waves in
// flight, than one item per wave.)
struct PQueue {
    const WorkItem* items[3];   // the work list of each pass
    int n[3];                   // its item count
    const int* total;           // [3][n_blocks] items of a pass touching a block
    int* cnt;                   // [3][n_blocks] items done; total + 1 once finalized
    int* head;                  // the ticket counter (cleared by the staging kernel)
    int* err;                   // set when a wait gave up (this launch)
    int* sticky;                // the same, kept until the next radii call
    int n_blocks;
    int spin_limit;             // polls before a wait gives up
};

// Distinct blocks of an item: its i blocks [I, I + rows), then its j blocks
// [J0, J1) other than those (J0 >= I).
__device__ __forceinline__ int pq_nd(const WorkItem& w)
{
    return w.rows + max(0, w.J1 - max(w.J0, w.I + w.rows));
}
__device__ __forceinline__ int pq_block(const WorkItem& w, int k)
{
    return k < w.rows ? w.I + k : max(w.J0, w.I + w.rows) + (k - w.rows);
}

// Waits until every block of item w is ready in pass `pass`; false if a wait
// gave up (or another wave's did).
__device__ bool pq_wait(const PQueue& q, int pass, const WorkItem& w, int lane)
{
    const int nd = pq_nd(w);
    const int* cnt = q.cnt + (size_t)pass * q.n_blocks;
    const int* tot = q.total + (size_t)pass * q.n_blocks;
    for (int c = 0; c < nd; c += kTile) {
        const int k = c + lane;
        int X = 0, want = 0;
        bool ok = k >= nd;
        if (!ok) {
            X = w.blk0 + pq_block(w, k);
            want = tot[X] + 1;
            ok = ld_dev(cnt + X) == want;
        }
        int spins = 0;
        while (__builtin_amdgcn_ballot_w64(!ok) != 0ull) {
            if (spins++ >= q.spin_limit || ld_dev(q.err) != 0) return false;
            __builtin_amdgcn_s_sleep(1);
            if (!ok) ok = ld_dev(cnt + X) == want;
        }
    }
    return true;
}

// Counts item w done on its blocks in pass `pass`; for every block this
// completes, fin(local block) finalizes it and the block is marked ready.
template <class Fin>
__device__ __forceinline__ void pq_complete(const PQueue& q, int pass, const WorkItem& w, int lane,
                                            Fin&& fin)
{
    // every fixed-point atomic of the item is performed before its blocks are
    // counted (vmcnt covers stores and atomics on gfx9)
    __builtin_amdgcn_s_waitcnt(0x0f70);       // vmcnt(0)
    const int nd = pq_nd(w);
    int* cnt = q.cnt + (size_t)pass * q.n_blocks;
    const int* tot = q.total + (size_t)pass * q.n_blocks;
    for (int c = 0; c < nd; c += kTile) {
        const int k = c + lane;
        int Lb = 0;
        bool last = false;
        if (k < nd) {
            Lb = pq_block(w, k);
            const int X = w.blk0 + Lb;
            last = atomicAdd(cnt + X, 1) == tot[X] - 1;
        }
        unsigned long long m = __builtin_amdgcn_ballot_w64(last);
        while (m != 0ull) {
            const int src = __builtin_ctzll(m);
            m &= m - 1ull;
            const int L = __builtin_amdgcn_readlane(Lb, src);
            fin(L);
            // the block's finals are visible device-wide before it is marked ready
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0) atomicAdd(cnt + w.blk0 + L, 1);
        }
    }
}

// LDS bytes per wave: the largest of the three passes' slices.
template <typename T>
struct PLds {
    static constexpr int radii = 2 * kTile * (int)sizeof(Q4<T>) + 2 * kTile * (int)sizeof(T) +
                                 kTile * 8 + kTile * 4;
    static constexpr int energy = 2 * kTile * (int)sizeof(Q4<T>) + 4 * kTile * (int)sizeof(T);
    static constexpr int chain = 4 * kTile * (int)sizeof(Q4<T>) + 4 * kTile * 8 + kTile * 4;
    static constexpr int bytes = radii > energy ? (radii > chain ? radii : chain)
                                                : (energy > chain ? energy : chain);
};

template <typename T, int W, int P0, int P1, bool GRAD, bool SALT, bool ONE>
__global__ __launch_bounds__(kTile * W) void k_pairs_queue(
    PQueue q, const T* __restrict__ RHO, GBConst c, T kC, T kT, SaltK<T> sk, Work<T> wk,
    T* __restrict__ born_R)
{
    __shared__ __align__(16) unsigned char lds_w[W][PLds<T>::bytes];
    __shared__ int ticket;
    const int wave = threadIdx.x / kTile, lane = threadIdx.x % kTile;
    if (threadIdx.x == 0) ticket = atomicAdd(q.head, 1);
    __syncthreads();
    int ntot = 0;
#pragma unroll
    for (int p = P0; p <= P1; ++p) ntot += q.n[p];
    // wave-uniform (scalar registers): the item and everything derived from it
    const int idx = __builtin_amdgcn_readfirstlane(ticket * W + wave);
    if (idx >= ntot) return;
    int p = P0, loc = idx;
    while (p < P1 && loc >= q.n[p]) { loc -= q.n[p]; ++p; }
    const WorkItem w = q.items[p][loc];
    if (p > P0 && !pq_wait(q, p - 1, w, lane)) {
        if (lane == 0) {
            atomicOr(q.err, 1);
            atomicOr(q.sticky, 1);
        }
        return;
    }
    unsigned char* lds = lds_w[wave];
    Q4<T>* sj = reinterpret_cast<Q4<T>*>(lds);
    if (P0 == 0 && p == 0) {
        T* sS = reinterpret_cast<T*>(sj + 2 * kTile);
        unsigned long long* sdef = reinterpret_cast<unsigned long long*>(sS + 2 * kTile);
        int* slist = reinterpret_cast<int*>(sdef + kTile);
        radii_item<T, 1, false>(w, lane, sj, sS, sdef, slist, wk.P, wk.Gx, wk.I_fx, wk.ovf, 0ull,
                                T(0), wk.box);
        pq_complete(q, 0, w, lane, [&](int L) {
            const int i = L * kTile + lane;
            if (i < w.n) radii_final_atom<T>(w.base + i, RHO, c, wk, born_R);
        });
    } else if (P0 <= 1 && P1 >= 1 && p == 1) {
        const CutK<T> ck{T(0), T(0)};
        T* sR = reinterpret_cast<T*>(sj + 2 * kTile);
        T* sA = sR + 2 * kTile;
        if (sizeof(T) == 4 && w.rows == 2)
            energy_item<T, GRAD, sizeof(T) == 4 ? 2 : 1, SALT, false, ONE>(
                w, lane, sj, sR, sA, wk.P, wk.R_t, wk.a_t, kC, kT, sk, ck, wk, 0ull);
        else
            energy_item<T, GRAD, 1, SALT, false, ONE>(w, lane, sj, sR, sA, wk.P, wk.R_t, wk.a_t,
                                                      kC, kT, sk, ck, wk, 0ull);
        // when the chain pass follows, the energy pass marks its blocks ready
        // (the chain pass forms B from their final G sums)
        if (P1 == 2) pq_complete(q, 1, w, lane, [&](int) {});
    } else if (P1 == 2 && p == 2) {
        Q4<T>* sb = sj + 2 * kTile;
        unsigned long long* sdef = reinterpret_cast<unsigned long long*>(sb + 2 * kTile);
        int* slist = reinterpret_cast<int*>(sdef + 4 * kTile);
        if (sizeof(T) == 4 && w.rows == 2)
            chain_item<T, sizeof(T) == 4 ? 2 : 1, false, ONE>(w, lane, sj, sb, sdef, slist, wk.P,
                                                            wk.Gx, wk, T(0), 0ull);
        else
            chain_item<T, 1, false, ONE>(w, lane, sj, sb, sdef, slist, wk.P, wk.Gx, wk,
                                         T(0), 0ull);
    }
}

// After the chain pass (three launches, or the queued launch): blocks
// [0, n_sum) sum the atoms' fixed-point energy shares of one system each
// (integer sums, order independent); the following blocks write one atom's
// outputs per thread: dE/dq, the forces and dE/drho (caller order).
//   dE/drho_k = G_k R_k^2 (1/rt_k^2 - T_k/rho_k^2) + B_k I_k + (pair part)
template <typename T>
__global__ __launch_bounds__(256) void k_post(int n_atoms, int n_sum, Work<T> w,
                                              double* __restrict__ e_coul,
                                              double* __restrict__ e_gb, T* __restrict__ dEdq,
                                              T* __restrict__ force, T* __restrict__ dEdrho,
                                              const T* __restrict__ RHO, double offset)
{
    const int t = threadIdx.x;
    if ((int)blockIdx.x < n_sum) {
        __shared__ long long part[2][4];
        const int b = blockIdx.x, lane = t % kTile, wave = t / kTile;
        long long s0 = 0, s1 = 0;
        for (int g = w.atom_offset[b] + t; g < w.atom_offset[b + 1]; g += 256) {
            s0 += (long long)w.EA_fx[g];
            s1 += (long long)w.EA_fx[w.n_atoms + g];
        }
#pragma unroll
        for (int o = kTile / 2; o > 0; o >>= 1) {
            s0 += __shfl_xor(s0, o);
            s1 += __shfl_xor(s1, o);
        }
        if (lane == 0) { part[0][wave] = s0; part[1][wave] = s1; }
        __syncthreads();
        if (t == 0) {
            long long ec = part[0][0] + part[0][1] + part[0][2] + part[0][3];
            long long eg = part[1][0] + part[1][1] + part[1][2] + part[1][3];
            if (e_coul) e_coul[b] = (double)ec * (1.0 / kScaleE);
            if (e_gb) e_gb[b] = (double)eg * (1.0 / kScaleE);
        }
        return;
    }
    const int k = ((int)blockIdx.x - n_sum) * 256 + t;
    if (k >= n_atoms) return;
    const int g = w.perm[k];
    if (dEdq) dEdq[g] = (T)((double)(long long)w.phi_fx[k] * (1.0 / kScaleF));
    if (force) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
            force[3 * (size_t)g + a] = (T)((double)(long long)w.F_fx[a * w.n_atoms + k] * (1.0 / kScaleF));
    }
    if (dEdrho) {
        double rho = (double)RHO[g];
        double rt = rho - offset;
        double R = w.R64[g];
        // G = dE/dR from its fixed-point sum and the chain weight B = G dR/dPsi
        const double G = (double)(long long)w.G_fx[k] * (1.0 / kScaleF);
        const double B = G * w.dRdPsi64[g];
        double v = G * R * R * (1.0 / (rt * rt) - w.T64[g] / (rho * rho))
                 + B * w.I64[g]
                 + (double)(long long)w.drho_fx[k] * (1.0 / kScaleF);
        dEdrho[g] = (T)v;
    }
}

// ============================================================ Monte Carlo
// Delta E_elec needs the potential phi_i on every site atom in FP64: a row pass
// over all atoms of the system, split in short chunks (many waves in flight);
// each chunk's FP64 partial is added in 2^-44 fixed point, so the sum does not
// depend on the order (deterministic) and k_site_dE reads one value per atom.

// k d(f), the GB factor of a pair term or a self term (f = R): kT = k (1/eps_in
// - 1/eps_out) without salt, k (1/eps_in - exp(-kappa f)/eps_out) with
// (kO = k/eps_out, kap = kappa).
__device__ __forceinline__ double gb_kd(double f, double kC, double kT, double kO, double kap)
{
    return kap == 0.0 ? kT : kC - kO * exp(-kap * f);
}

// k/(eps_in r) - k d(f) / f_GB for one pair (FP64); a = 1/(2R); 0 at or beyond
// the pair cutoff (cut2 = cutoff^2, infinite for none).
__device__ __forceinline__ double pairK(double dx, double dy, double dz, double Ra, double aa,
                                        double Rb, double ab, double kC, double kT, double kO,
                                        double kap, double cut2)
{
    double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 >= cut2) return 0.0;
    double invr = rsq64(r2);
    double ex = exp(-r2 * (aa * ab));
    double f2 = fma(Ra * Rb, ex, r2);
    double invf = rsq64(f2);
    return kC * invr - gb_kd(f2 * invf, kC, kT, kO, kap) * invf;
}

// One lane per site atom.  The chunk's j atoms (positions and radii of the
// last gb_radii call, current charges) are staged into LDS by the first
// kPhiChunk lanes with one load each, then read as wave-uniform broadcasts.
template <typename T>
__global__ __launch_bounds__(kTile) void k_site_phi_rows(
    const RowItem* __restrict__ items, const int32_t* __restrict__ site_atoms,
    const Row64* __restrict__ rows, const T* __restrict__ Q, double kC, double kT, double kO,
    double kap, double cut2,
    unsigned long long* __restrict__ phi_fx, int* __restrict__ ovf)
{
    __shared__ double2 s_xy[kPhiChunk], s_zR[kPhiChunk], s_Aq[kPhiChunk];
    const RowItem w = items[blockIdx.x];
    const int lane = threadIdx.x;
    const int sa = w.sa0 + lane;
    const bool v = sa < w.sa1;
    const int gi = v ? site_atoms[sa] : w.base;
    const int nj = w.j1 - w.j0;                    // 1 .. kPhiChunk
    if (lane < nj) {
        const int gj = w.base + w.j0 + lane;
        const Row64 r = rows[gj];
        s_xy[lane] = make_double2(r.x, r.y);
        s_zR[lane] = make_double2(r.z, r.R);
        s_Aq[lane] = make_double2(r.A, (double)Q[gj]);
    }
    const Row64 ri = rows[gi];
    const int self = gi - (w.base + w.j0);         // this lane's own atom, if in the chunk
    __syncthreads();
    double acc = 0.0;
#pragma unroll 4
    for (int k = 0; k < nj; ++k) {
        const double2 xy = s_xy[k], zR = s_zR[k], Aq = s_Aq[k];
        double K = pairK(ri.x - xy.x, ri.y - xy.y, ri.z - zR.x, ri.R, ri.A, zR.y, Aq.x, kC, kT, kO, kap, cut2);
        acc += (k == self) ? 0.0 : Aq.y * K;
    }
    bool bad = false;
    const long long f = to_fixed(acc, kScaleP, bad);
    if (v) fx_add(&phi_fx[w.out + lane], f);
    if (bad) *ovf = 1;
}

__global__ void k_clear64(unsigned long long* __restrict__ p, int n)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0ull;
}

// Deterministic sum of NV doubles over a block of NW wavefronts: a fixed
// butterfly inside each wavefront, then the wave sums in wave order.  Every
// thread receives the totals.
template <int NV, int NW>
__device__ void block_sum(double (*buf)[NW], double* v)
{
    const int t = threadIdx.x, lane = t % kTile, wave = t / kTile;
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        double x = v[a];
#pragma unroll
        for (int off = kTile / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
        v[a] = x;
    }
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < NV; ++a) buf[a][wave] = v[a];
    }
    __syncthreads();
    // thread a adds the wave sums of value a in wave order
    if (t < NV) {
        double x = buf[t][0];
#pragma unroll 1
        for (int k = 1; k < NW; ++k) x += buf[t][k];
        buf[t][0] = x;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NV; ++a) v[a] = buf[a][0];
    __syncthreads();
}

constexpr int kMC = 256;    // threads of the per-system Monte Carlo step
// threads of the per-site Delta E kernel: four waves (a site's triangle of
// atom pairs is short, and a small workgroup finds room on the CUs beside the
// force passes sooner than one of 16 waves: 7 us shorter E-REMD step)
constexpr int kSDE = 256;
constexpr int kSweep = 1024;  // threads of the per-system sweep kernel (16 waves on one CU)

template <typename T>
__global__ __launch_bounds__(kSDE) void k_site_dE(
    SiteDev sd, const T* __restrict__ X, const T* __restrict__ Y, const T* __restrict__ Z,
    const T* __restrict__ Q, const double* __restrict__ R64, const double* __restrict__ A64,
    double kC, double kT, double kO, double kap, double cut2,
    const unsigned long long* __restrict__ phi_fx,
    const int32_t* __restrict__ current_state,
    const double* __restrict__ pH, const double* __restrict__ E_volt, double T_kelvin,
    double* __restrict__ dE, double* __restrict__ dG)
{
    __shared__ double sx[kMaxSiteAtoms], sy[kMaxSiteAtoms], sz[kMaxSiteAtoms], sR[kMaxSiteAtoms];
    __shared__ double sA[kMaxSiteAtoms];
    __shared__ double sphi[kMaxSiteAtoms];
    __shared__ double sdq[kMaxStates - 1][kMaxSiteAtoms];
    __shared__ double red[2 * (kMaxStates - 1)][kSDE / kTile];
    const int m = blockIdx.x;
    const int t = threadIdx.x;
    const int a0 = sd.site_atom_offset[m];
    const int na = sd.site_atom_offset[m + 1] - a0;
    const int g0 = sd.site_state_offset[m];
    const int ns = sd.site_state_offset[m + 1] - g0;
    const int cur = current_state[m];
    const int nc = ns - 1;
    const int sa_site0 = sd.site_sa_offset[m];
    const double* qcur = sd.state_charges + sd.state_charge_offset[g0 + cur];
    for (int a = t; a < na; a += kSDE) {
        int g = sd.site_atoms[a0 + a];
        double R = R64[g];
        sx[a] = X[g]; sy[a] = Y[g]; sz[a] = Z[g]; sR[a] = R; sA[a] = A64[g];
        double phi = -gb_kd(R, kC, kT, kO, kap) * (double)Q[g] / R;   // self term
        phi += (double)(long long)phi_fx[sa_site0 + a] * (1.0 / kScaleP);
        sphi[a] = phi;
        for (int c = 0; c < nc; ++c) {
            int s_new = c < cur ? c : c + 1;
            sdq[c][a] = sd.state_charges[sd.state_charge_offset[g0 + s_new] + a] - qcur[a];
        }
    }
    __syncthreads();
    double part[2 * (kMaxStates - 1)];
#pragma unroll
    for (int c = 0; c < 2 * (kMaxStates - 1); ++c) part[c] = 0.0;
    // linear term
    for (int a = t; a < na; a += kSDE) {
#pragma unroll
        for (int c = 0; c < kMaxStates - 1; ++c)
            if (c < nc) part[c] += sdq[c][a] * sphi[a];
    }
    // quadratic term over the triangle b >= a (diagonal once, off-diagonal
    // pairs twice); triangle index p = b (b + 1) / 2 + a
    const int n_tri = na * (na + 1) / 2;
#pragma unroll 1
    for (int p = t; p < n_tri; p += kSDE) {
        int b = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
        b += (b + 1) * (b + 2) / 2 <= p;          // guard the rounding of the root
        b -= b * (b + 1) / 2 > p;
        const int a = p - b * (b + 1) / 2;
        double K = (a == b) ? -gb_kd(sR[a], kC, kT, kO, kap) / sR[a]
                            : 2.0 * pairK(sx[a] - sx[b], sy[a] - sy[b], sz[a] - sz[b], sR[a], sA[a],
                                          sR[b], sA[b], kC, kT, kO, kap, cut2);
#pragma unroll
        for (int c = 0; c < kMaxStates - 1; ++c)
            if (c < nc) part[kMaxStates - 1 + c] += sdq[c][a] * sdq[c][b] * K;
    }
    block_sum<2 * (kMaxStates - 1), kSDE / kTile>(red, part);
    double lin = 0.0, quad = 0.0;
#pragma unroll
    for (int c = 0; c < kMaxStates - 1; ++c)
        if (c == t) { lin = part[c]; quad = part[kMaxStates - 1 + c]; }
    if (t < nc) {
        int c = t;
        int s_new = c < cur ? c : c + 1;
        double de = lin + 0.5 * quad;
        int cand = sd.cand_offset[m] + c;
        dE[cand] = de;
        if (dG) {
            int b = sd.site_system[m];
            double drive = sd.site_kind[m] == 0 ? kKB * T_kelvin * kLn10 * pH[b] : kFaraday * E_volt[b];
            dG[cand] = de + drive * (double)(sd.state_count[g0 + s_new] - sd.state_count[g0 + cur])
                     - (sd.state_gref[g0 + s_new] - sd.state_gref[g0 + cur]);
        }
    }
}

__device__ __forceinline__ int pick_index(double u, int n)
{
    int k = (int)floor(u * (double)n);
    return k < n - 1 ? (k < 0 ? 0 : k) : n - 1;
}

template <typename T>
__global__ __launch_bounds__(kMC) void k_mc_step(
    SiteDev sd, const T* __restrict__ X, const T* __restrict__ Y, const T* __restrict__ Z,
    T* __restrict__ Q, const double* __restrict__ R64, const double* __restrict__ A64, double kC,
    double kT, double kO, double kap, double cut2, int32_t* __restrict__ current_state,
    const double* __restrict__ pH,
    const double* __restrict__ E_volt, double T_kelvin, const double* __restrict__ dEin,
    const double* __restrict__ dGin, const double* __restrict__ u,
    int32_t* __restrict__ n_electrons, int64_t* __restrict__ counters,
    int32_t* __restrict__ accepted)
{
    __shared__ double red[1][4];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    const double* ub = u + 6 * (size_t)b;
    const double kTB = kKB * T_kelvin;
    int acc_p = 0, m_p = -1, s_p = 0, snew_p = 0;
    // ---- protonation attempt
    {
        const int p0 = sd.sys_prot_offset[b], np = sd.sys_prot_offset[b + 1] - p0;
        if (np > 0) {
            m_p = sd.sys_prot_sites[p0 + pick_index(ub[0], np)];
            const int g0 = sd.site_state_offset[m_p];
            const int ns = sd.site_state_offset[m_p + 1] - g0;
            s_p = current_state[m_p];
            const int tp = pick_index(ub[1], ns - 1);
            snew_p = tp < s_p ? tp : tp + 1;
            const double dg = dGin[sd.cand_offset[m_p] + tp];
            acc_p = ub[2] < exp(-dg / kTB) ? 1 : 0;
        }
    }
    // ---- redox attempt, on the charges left by the protonation attempt
    int acc_r = 0, m_r = -1, s_r = 0, snew_r = 0;
    {
        const int r0 = sd.sys_redox_offset[b], nr = sd.sys_redox_offset[b + 1] - r0;
        if (nr > 0) {
            m_r = sd.sys_redox_sites[r0 + pick_index(ub[3], nr)];
            const int g0 = sd.site_state_offset[m_r];
            const int ns = sd.site_state_offset[m_r + 1] - g0;
            s_r = current_state[m_r];
            const int tp = pick_index(ub[4], ns - 1);
            snew_r = tp < s_r ? tp : tp + 1;
            double dg = dGin[sd.cand_offset[m_r] + tp];
            if (acc_p) {
                // cross term dq_redox . K . dq_prot (sites are disjoint)
                const int ar0 = sd.site_atom_offset[m_r], nar = sd.site_atom_offset[m_r + 1] - ar0;
                const int ap0 = sd.site_atom_offset[m_p], nap = sd.site_atom_offset[m_p + 1] - ap0;
                const int gp0 = sd.site_state_offset[m_p];
                const double* qr1 = sd.state_charges + sd.state_charge_offset[g0 + snew_r];
                const double* qr0 = sd.state_charges + sd.state_charge_offset[g0 + s_r];
                const double* qp1 = sd.state_charges + sd.state_charge_offset[gp0 + snew_p];
                const double* qp0 = sd.state_charges + sd.state_charge_offset[gp0 + s_p];
                double part[1] = {0.0};
                for (int p = t; p < nar * nap; p += kMC) {
                    int a = p / nap, c = p - a * nap;
                    int ga = sd.site_atoms[ar0 + a], gc = sd.site_atoms[ap0 + c];
                    double K = pairK((double)X[ga] - (double)X[gc], (double)Y[ga] - (double)Y[gc],
                                     (double)Z[ga] - (double)Z[gc], R64[ga], A64[ga], R64[gc],
                                     A64[gc], kC, kT, kO, kap, cut2);
                    part[0] += (qr1[a] - qr0[a]) * (qp1[c] - qp0[c]) * K;
                }
                block_sum<1, kMC / kTile>(red, part);
                dg += part[0];
            }
            acc_r = ub[5] < exp(-dg / kTB) ? 1 : 0;
        }
    }
    // ---- apply
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
        const int m = pass == 0 ? m_p : m_r;
        const int acc = pass == 0 ? acc_p : acc_r;
        const int snew = pass == 0 ? snew_p : snew_r;
        if (m < 0) continue;
        if (acc) {
            const int a0 = sd.site_atom_offset[m], na = sd.site_atom_offset[m + 1] - a0;
            const double* qn = sd.state_charges + sd.state_charge_offset[sd.site_state_offset[m] + snew];
            for (int a = t; a < na; a += kMC) Q[sd.site_atoms[a0 + a]] = (T)qn[a];
        }
        if (t == 0) {
            if (acc) current_state[m] = snew;
            if (counters) {
                counters[2 * (size_t)m] += 1;
                counters[2 * (size_t)m + 1] += acc;
            }
        }
    }
    if (t == 0) {
        if (accepted) { accepted[2 * b] = acc_p; accepted[2 * b + 1] = acc_r; }
        if (n_electrons) {
            const int r0 = sd.sys_redox_offset[b], nr = sd.sys_redox_offset[b + 1] - r0;
            int ne = 0;
            for (int k = 0; k < nr; ++k) {
                int m = sd.sys_redox_sites[r0 + k];
                int st = (m == m_r && acc_r) ? snew_r : current_state[m];
                ne += sd.state_count[sd.site_state_offset[m] + st];
            }
            n_electrons[b] = ne;
        }
    }
}

// Sequential sweep (section III.A.2): one workgroup per system visits every
// site of the requested kinds once, protonation sites first, each kind in the
// order of ascending u[3m] (ties by site index).  The FP64 potentials of all
// the system's site atoms live in LDS (dynamic, [6][n_sa]: x, y, z, R, A,
// phi); a visit computes Delta E = dq . phi + 1/2 dq . K_SS . dq from them,
// and an accepted change adds K dq to every site atom's potential, so the
// next visit sees the charges it left.  All threads evaluate the same
// block-reduced Delta G and so take the same decision.
template <typename T>
__global__ __launch_bounds__(kSweep) void k_mc_sweep(
    SiteDev sd, const T* __restrict__ X, const T* __restrict__ Y, const T* __restrict__ Z,
    const T* __restrict__ Q, T* __restrict__ Qout, const double* __restrict__ R64,
    const double* __restrict__ A64, double kC, double kT, double kO, double kap, double cut2,
    const unsigned long long* __restrict__ phi_fx, int32_t* __restrict__ current_state,
    const double* __restrict__ pH, const double* __restrict__ E_volt, double T_kelvin, int kinds,
    const double* __restrict__ u, int32_t* __restrict__ n_electrons,
    int64_t* __restrict__ counters, int32_t* __restrict__ accepted, double* __restrict__ dG_out)
{
    extern __shared__ double s_sa[];
    __shared__ double sdq[kMaxSiteAtoms];
    __shared__ int order[kMaxSweepSites];
    __shared__ double red[2][kSweep / kTile];
    const int b = blockIdx.x, t = threadIdx.x;
    const int sa0 = sd.sys_sa_offset[b], nsa = sd.sys_sa_offset[b + 1] - sa0;
    double* sx = s_sa;
    double* sy = sx + nsa;
    double* sz = sy + nsa;
    double* sR = sz + nsa;
    double* sA = sR + nsa;
    double* sphi = sA + nsa;
    for (int a = t; a < nsa; a += kSweep) {
        const int g = sd.site_atoms[sa0 + a];
        const double R = R64[g];
        sx[a] = X[g]; sy[a] = Y[g]; sz[a] = Z[g];
        sR[a] = R; sA[a] = A64[g];
        sphi[a] = (double)(long long)phi_fx[sa0 + a] * (1.0 / kScaleP)
                - gb_kd(R, kC, kT, kO, kap) * (double)Q[g] / R;
    }
    const double kTB = kKB * T_kelvin;
    for (int kind = 0; kind < 2; ++kind) {
        if (!(kinds & (1 << kind))) continue;
        const int o0 = kind == 0 ? sd.sys_prot_offset[b] : sd.sys_redox_offset[b];
        const int cnt = (kind == 0 ? sd.sys_prot_offset[b + 1] : sd.sys_redox_offset[b + 1]) - o0;
        const int32_t* list = (kind == 0 ? sd.sys_prot_sites : sd.sys_redox_sites) + o0;
        __syncthreads();
        // rank of each site by (u[3m], m); a NaN key sorts last, so the ranks
        // always form a permutation
        auto order_key = [&](int m) {
            const double k = u[3 * (size_t)m];
            return k == k ? k : 2.0;
        };
        for (int k = t; k < cnt; k += kSweep) {
            const int m = list[k];
            const double key = order_key(m);
            int rank = 0;
            for (int j = 0; j < cnt; ++j) {
                const int mj = list[j];
                const double kj = order_key(mj);
                rank += (kj < key) || (kj == key && mj < m);
            }
            order[rank] = m;
        }
        __syncthreads();
        const double drive = kind == 0 ? kKB * T_kelvin * kLn10 * pH[b] : kFaraday * E_volt[b];
        for (int v = 0; v < cnt; ++v) {
            const int m = order[v];
            const int a0 = sd.site_atom_offset[m] - sa0;
            const int na = sd.site_atom_offset[m + 1] - sd.site_atom_offset[m];
            const int g0 = sd.site_state_offset[m];
            const int ns = sd.site_state_offset[m + 1] - g0;
            const int s = current_state[m];
            const int tp = pick_index(u[3 * (size_t)m + 1], ns - 1);
            const int s_new = tp < s ? tp : tp + 1;
            const double* qn = sd.state_charges + sd.state_charge_offset[g0 + s_new];
            const double* qo = sd.state_charges + sd.state_charge_offset[g0 + s];
            for (int a = t; a < na; a += kSweep) sdq[a] = qn[a] - qo[a];
            __syncthreads();
            double part[2] = {0.0, 0.0};
            for (int a = t; a < na; a += kSweep) part[0] += sdq[a] * sphi[a0 + a];
            const int n_tri = na * (na + 1) / 2;
#pragma unroll 1
            for (int p = t; p < n_tri; p += kSweep) {
                int c = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
                c += (c + 1) * (c + 2) / 2 <= p;
                c -= c * (c + 1) / 2 > p;
                const int a = p - c * (c + 1) / 2;
                const int ia = a0 + a, ic = a0 + c;
                const double K = (a == c) ? -gb_kd(sR[ia], kC, kT, kO, kap) / sR[ia]
                                          : 2.0 * pairK(sx[ia] - sx[ic], sy[ia] - sy[ic], sz[ia] - sz[ic],
                                                        sR[ia], sA[ia], sR[ic], sA[ic], kC, kT, kO, kap, cut2);
                part[1] += sdq[a] * sdq[c] * K;
            }
            block_sum<2, kSweep / kTile>(red, part);
            const double dE = part[0] + 0.5 * part[1];
            const double dg = dE + drive * (double)(sd.state_count[g0 + s_new] - sd.state_count[g0 + s])
                            - (sd.state_gref[g0 + s_new] - sd.state_gref[g0 + s]);
            const bool acc = u[3 * (size_t)m + 2] < exp(-dg / kTB);
            if (t == 0) {
                if (accepted) accepted[m] = acc ? 1 : 0;
                if (dG_out) dG_out[m] = dg;
                if (counters) {
                    counters[2 * (size_t)m] += 1;
                    counters[2 * (size_t)m + 1] += acc ? 1 : 0;
                }
                if (acc) current_state[m] = s_new;
            }
            if (acc) {
                // every site atom's potential gains K dq of this site
                for (int i = t; i < nsa; i += kSweep) {
                    double d = 0.0;
                    for (int c = 0; c < na; ++c) {
                        const int ic = a0 + c;
                        d += sdq[c] * (i == ic ? -gb_kd(sR[i], kC, kT, kO, kap) / sR[i]
                                               : pairK(sx[i] - sx[ic], sy[i] - sy[ic], sz[i] - sz[ic],
                                                       sR[i], sA[i], sR[ic], sA[ic], kC, kT, kO, kap, cut2));
                    }
                    sphi[i] += d;
                }
                for (int a = t; a < na; a += kSweep) Qout[sd.site_atoms[sa0 + a0 + a]] = (T)qn[a];
            }
            __syncthreads();
        }
    }
    if (t == 0 && n_electrons) {
        const int r0 = sd.sys_redox_offset[b], nr = sd.sys_redox_offset[b + 1] - r0;
        int ne = 0;
        for (int k = 0; k < nr; ++k) {
            const int m = sd.sys_redox_sites[r0 + k];
            ne += sd.state_count[sd.site_state_offset[m] + current_state[m]];
        }
        n_electrons[b] = ne;
    }
}

// E-REMD exchange: one workgroup; pairs are disjoint so they update in parallel.
__global__ __launch_bounds__(256) void k_remd_exchange(int M, const double* __restrict__ E_rung,
                                                       const int32_t* __restrict__ Ne,
                                                       int32_t* __restrict__ rep, double T_kelvin,
                                                       int parity, int wrap,
                                                       const double* __restrict__ u,
                                                       int32_t* __restrict__ accepted,
                                                       double* __restrict__ E_of_rep)
{
    const int n_inner = (M - parity) / 2;
    const int n_pairs = n_inner + ((parity == 1 && wrap && (M % 2 == 0) && M > 2) ? 1 : 0);
    const double beta = kFaraday / (kKB * T_kelvin);
    for (int p = threadIdx.x; p < n_pairs; p += blockDim.x) {
        int l, n2;
        if (p < n_inner) { l = parity + 2 * p; n2 = l + 1; }
        else { l = M - 1; n2 = 0; }
        int i = rep[l], j = rep[n2];
        // a malformed permutation never reads out of bounds: such a pair is not exchanged
        bool ok = (unsigned)i < (unsigned)M && (unsigned)j < (unsigned)M;
        double delta = ok ? beta * (E_rung[n2] - E_rung[l]) * (double)(Ne[i] - Ne[j]) : 0.0;
        int acc = (ok && (delta < 0.0 || u[p] < exp(-delta))) ? 1 : 0;
        if (acc) { rep[l] = j; rep[n2] = i; }
        if (accepted) accepted[p] = acc;
    }
    __syncthreads();
    if (E_of_rep)
        for (int l = threadIdx.x; l < M; l += blockDim.x)
            if ((unsigned)rep[l] < (unsigned)M) E_of_rep[rep[l]] = E_rung[l];
}

// ============================================================ launchers

// Squared pair cutoff of the FP64 Monte Carlo kernels (infinite for none).
static inline double cut2_of(const GBConst& c)
{
    return c.cutoff > 0.0 ? c.cutoff * c.cutoff : __builtin_huge_val();
}

static inline int blocks_for(size_t n, int bs) { return (int)((n + bs - 1) / bs); }

// Launch of a kernel that the timing hook measures.  With the hook on (ev not
// NULL) the start and stop events are bound to the dispatch itself, so their
// interval is the kernel's own execution, without queue gaps.
#define GBMC_LAUNCH_TIMED(ev, id, K, grid, block, s, ...)                                      \
    do {                                                                                       \
        if (ev)                                                                                \
            hipExtLaunchKernelGGL(K, grid, block, 0, s, (ev)[2 * (id)], (ev)[2 * (id) + 1], 0, \
                                  __VA_ARGS__);                                                \
        else                                                                                   \
            hipLaunchKernelGGL(K, grid, block, 0, s, __VA_ARGS__);                             \
    } while (0)

// Pair-kernel launch with W independent wavefronts per workgroup.
#define GBMC_DISPATCH_W(W_, CALL)             \
    switch (W_) {                             \
    case 1: { constexpr int W = 1; CALL; } break; \
    case 2: { constexpr int W = 2; CALL; } break; \
    case 4: { constexpr int W = 4; CALL; } break; \
    default: { constexpr int W = 8; CALL; } break; \
    }

// Block bounds and the compacted work of the cutoff passes (positions as
// staged by the caller of this function).
template <typename T>
static void launch_cut_lists(const CutPlan& cp, const GBConst& c, const Work<T>& w, hipStream_t s)
{
    if (cp.n_blocks == 0) return;
    hipLaunchKernelGGL(k_block_bounds<T>, dim3(blocks_for(cp.n_blocks, 4)), dim3(256), 0, s,
                       cp.blocks, cp.n_blocks, w.P, w.Gx, w.bnd, w.smax, w.ccount);
    if (cp.n_chunks > 0)
        hipLaunchKernelGGL(k_cut_items, dim3(blocks_for(cp.n_chunks, kCutWaves)),
                           dim3(kTile * kCutWaves), 0, s, cp.chunks, cp.n_chunks, w.bnd, w.smax,
                           (float)c.rgbmax, (float)c.cutoff, w.citems[0], w.citems[1], w.ccount,
                           w.cut_cap);
}

// Workgroups of a grid-stride cutoff pass: enough waves to fill the chip.
static inline int cut_groups(int cap, int W)
{
    return std::max(1, std::min(blocks_for(cap, W), 16384 / W));
}

template <typename T>
hipError_t launch_radii(const WorkItem* items, int n_items, int wpg, int n_atoms,
                        const CutPlan& cp,
                        const T* x, const T* y, const T* z, const T* rho, const T* screen,
                        const GBConst& c, const Work<T>& w, T* born_R, hipStream_t s,
                        hipEvent_t* ev, const T* q)
{
    if (n_atoms == 0) return hipSuccess;
    // staging also clears I_fx and the overflow flags: every evaluation starts
    // at zero.  With charges (q not NULL: the full evaluation, whose energy
    // pass then stages nothing) it also packs them and clears the accumulators
    // of the energy and chain passes ([8][N] from F_fx on).
    StageClear zc{};
    zc.acc0 = w.I_fx; zc.n_acc0 = 1;
    zc.f0 = w.ovf; zc.n_f0 = 2;
    if (q) { zc.acc1 = w.F_fx; zc.n_acc1 = 8; }
    hipLaunchKernelGGL(k_stage<T>, dim3(blocks_for(cp.n_blocks, 4)), dim3(256), 0, s, cp.blocks,
                       cp.n_blocks, n_atoms, w.perm, x, y, z, q, rho, screen,
                       (T)c.offset, w.P, w.Gx, w.box, zc);
    if (c.rgbmax > 0.0 || c.cutoff > 0.0) launch_cut_lists<T>(cp, c, w, s);
    if (n_items > 0) {
        if (c.rgbmax > 0.0)
            GBMC_DISPATCH_W(wpg, GBMC_LAUNCH_TIMED(ev, kKRadii, (k_radii_pairs<T, W, true>),
                                                   dim3(cut_groups(w.cut_cap, W)), dim3(kTile * W),
                                                   s, items, n_items, w.citems[0], w.ccount, w.P,
                                                   w.Gx, w.I_fx, w.ovf, (T)c.rgbmax, w.box))
        else
            GBMC_DISPATCH_W(wpg, GBMC_LAUNCH_TIMED(ev, kKRadii, (k_radii_pairs<T, W, false>),
                                                   dim3(blocks_for(n_items, W)), dim3(kTile * W), s,
                                                   items, n_items, w.citems[0], w.ccount, w.P,
                                                   w.Gx, w.I_fx, w.ovf, (T)0, w.box))
    }
    hipLaunchKernelGGL(k_radii_finalize<T>, dim3(blocks_for(n_atoms, 256)), dim3(256), 0, s, n_atoms,
                       rho, c, w, born_R);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_energy_forces(const PassShape& pe, const PassShape& pc, int n_atoms, int n_sys,
                                const CutPlan& cp,
                                const T* x, const T* y, const T* z, const T* q, const T* rho,
                                const T* screen, const GBConst& c, const Work<T>& w,
                                double* e_coul, double* e_gb, T* force, T* dEdq, T* dEdrho,
                                hipStream_t s, hipEvent_t* ev, bool staged)
{
    const bool grad = force || dEdq || dEdrho;
    const bool chain = force || dEdrho;
    // positions and charges as given to this call, in processing order; F, G,
    // phi, drho and the two energy shares ([8][N] from F_fx on) cleared
    // alongside (staged: the full evaluation's radii staging did both)
    if (n_atoms > 0 && !staged) {
        StageClear zc{};
        zc.acc0 = w.F_fx; zc.n_acc0 = 8;
        hipLaunchKernelGGL(k_stage<T>, dim3(blocks_for(cp.n_blocks, 4)), dim3(256), 0, s,
                           cp.blocks, cp.n_blocks, n_atoms, w.perm, x, y, z, q, rho, screen,
                           (T)c.offset, w.P, w.Gx, w.box, zc);
    }
    // block bounds and compacted work (positions as staged here, the same as
    // the preceding gb_radii call's)
    if (c.rgbmax > 0.0 || c.cutoff > 0.0) launch_cut_lists<T>(cp, c, w, s);
    if (pe.n_items > 0) {
        const SaltK<T> sk{(T)c.kO, (T)c.kappa, (T)(c.kappa * kLog2e)};
        const CutK<T> ck{(T)c.cutoff, (T)(c.cutoff * c.cutoff)};
#define GBMC_ENERGY_LAUNCH(G_, S_, C_, O_)                                                        \
    GBMC_DISPATCH_W(pe.waves_per_group,                                                          \
                    GBMC_LAUNCH_TIMED(ev, kKEnergy, (k_energy_pairs<T, G_, W, S_, C_, O_>),      \
                                      dim3(C_ ? cut_groups(w.cut_cap, W)                         \
                                              : blocks_for(pe.n_items, W)),                      \
                                      dim3(kTile * W), s,                                        \
                                      pe.items, pe.n_items, w.P, w.R_t, w.a_t, (T)c.kC, (T)c.kT, \
                                      sk, ck, w))
        const bool salt = c.kappa != 0.0, cut = c.cutoff > 0.0, one = pe.one_tile;
        if (grad) {
            if (salt) {
                if (cut) GBMC_ENERGY_LAUNCH(true, true, true, false)
                else if (one) GBMC_ENERGY_LAUNCH(true, true, false, true)
                else GBMC_ENERGY_LAUNCH(true, true, false, false)
            } else {
                if (cut) GBMC_ENERGY_LAUNCH(true, false, true, false)
                else if (one) GBMC_ENERGY_LAUNCH(true, false, false, true)
                else GBMC_ENERGY_LAUNCH(true, false, false, false)
            }
        } else {
            if (salt) {
                if (cut) GBMC_ENERGY_LAUNCH(false, true, true, false)
                else if (one) GBMC_ENERGY_LAUNCH(false, true, false, true)
                else GBMC_ENERGY_LAUNCH(false, true, false, false)
            } else {
                if (cut) GBMC_ENERGY_LAUNCH(false, false, true, false)
                else if (one) GBMC_ENERGY_LAUNCH(false, false, false, true)
                else GBMC_ENERGY_LAUNCH(false, false, false, false)
            }
        }
#undef GBMC_ENERGY_LAUNCH
    }
    const int n_sum = (e_coul || e_gb) ? n_sys : 0;
    const int n_fin = grad ? blocks_for(n_atoms, 256) : 0;
    // without the chain pass the energies and dE/dq are written here; with it
    // the chain pass forms B from the G sums itself and k_post writes every
    // output at the end (one launch fewer between the pair passes)
    if (!chain && n_sum + n_fin > 0)
        hipLaunchKernelGGL(k_energy_finalize<T>, dim3(n_sum + n_fin), dim3(256), 0, s, n_atoms, n_sum,
                           w, e_coul, e_gb, dEdq, grad);
    if (chain && pc.n_items > 0) {
        if (c.rgbmax > 0.0)
            GBMC_DISPATCH_W(pc.waves_per_group,
                            GBMC_LAUNCH_TIMED(ev, kKChain, (k_chain_pairs<T, W, true, false>),
                                              dim3(cut_groups(w.cut_cap, W)), dim3(kTile * W), s,
                                              pc.items, pc.n_items, w.P, w.Gx, w,
                                              (T)c.rgbmax))
        else if (pc.one_tile)
            GBMC_DISPATCH_W(pc.waves_per_group,
                            GBMC_LAUNCH_TIMED(ev, kKChain, (k_chain_pairs<T, W, false, true>),
                                              dim3(blocks_for(pc.n_items, W)), dim3(kTile * W), s,
                                              pc.items, pc.n_items, w.P, w.Gx, w, (T)0))
        else
            GBMC_DISPATCH_W(pc.waves_per_group,
                            GBMC_LAUNCH_TIMED(ev, kKChain, (k_chain_pairs<T, W, false, false>),
                                              dim3(blocks_for(pc.n_items, W)), dim3(kTile * W), s,
                                              pc.items, pc.n_items, w.P, w.Gx, w, (T)0))
    }
    if (chain && n_sum + n_fin > 0)
        hipLaunchKernelGGL(k_post<T>, dim3(n_sum + n_fin), dim3(256), 0, s, n_atoms, n_sum, w,
                           e_coul, e_gb, dEdq, force, dEdrho, rho, c.offset);
    return hipGetLastError();
}

constexpr int kPersistW = 8;     // waves per workgroup (items per ticket) of the queued launch

template <typename T, int P0, int P1, bool G, bool S, bool O>
static hipError_t queued_dispatch(const PQueue& pq, int ntot, const QueueShape& sh,
                                      const T* rho, const GBConst& c, const Work<T>& w, T* born_R,
                                      hipStream_t s, hipEvent_t* ev, int id)
{
    (void)sh;
    auto kern = k_pairs_queue<T, kPersistW, P0, P1, G, S, O>;
    const SaltK<T> sk{(T)c.kO, (T)c.kappa, (T)(c.kappa * kLog2e)};
    GBMC_LAUNCH_TIMED(ev, id, kern, dim3(blocks_for(ntot, kPersistW)), dim3(kTile * kPersistW), s,
                      pq, rho, c, (T)c.kC, (T)c.kT, sk, w, born_R);
    return hipGetLastError();
}

template <typename T, int P0, int P1>
static hipError_t queued_variant(bool salt, bool one, const PQueue& pq, int ntot,
                                 const QueueShape& sh, const T* rho, const GBConst& c,
                                 const Work<T>& w, T* born_R, hipStream_t s, hipEvent_t* ev, int id)
{
    if (salt)
        return one ? queued_dispatch<T, P0, P1, true, true, true>(pq, ntot, sh, rho, c, w, born_R, s, ev, id)
                   : queued_dispatch<T, P0, P1, true, true, false>(pq, ntot, sh, rho, c, w, born_R, s, ev, id);
    return one ? queued_dispatch<T, P0, P1, true, false, true>(pq, ntot, sh, rho, c, w, born_R, s, ev, id)
               : queued_dispatch<T, P0, P1, true, false, false>(pq, ntot, sh, rho, c, w, born_R, s, ev, id);
}

template <typename T>
hipError_t launch_queued(const QueueShape& sh, int n_atoms, int n_sys, const T* x, const T* y,
                         const T* z, const T* q, const T* rho, const T* screen, const GBConst& c,
                         const Work<T>& w, T* born_R, double* e_coul, double* e_gb, T* force,
                         T* dEdq, T* dEdrho, hipStream_t s, hipEvent_t* ev, int timing_id)
{
    if (n_atoms == 0) return hipSuccess;
    // staging: atoms packed in processing order; the accumulators, the
    // overflow flags, the ticket counter, the error word and the block
    // counters start at zero
    StageClear zc{};
    zc.acc0 = w.I_fx; zc.n_acc0 = 1;
    zc.acc1 = w.F_fx; zc.n_acc1 = 8;
    zc.f0 = w.ovf; zc.n_f0 = 2;
    zc.f1 = w.qhead; zc.n_f1 = kQueueWords;
    zc.cnt = w.qcnt; zc.n_cnt = 3 * sh.n_blocks;
    // (one wave per block: at least 256 threads, beyond the kQueueWords flags)
    hipLaunchKernelGGL(k_stage<T>, dim3(blocks_for(sh.n_blocks, 4)), dim3(256), 0, s, sh.blocks,
                       sh.n_blocks, n_atoms, w.perm, x, y, z, q, rho, screen, (T)c.offset, w.P,
                       w.Gx, w.box, zc);
    PQueue pq{};
    int ntot = 0;
    for (int k = 0; k < 3; ++k) {
        pq.items[k] = sh.items[k];
        pq.n[k] = sh.n_items[k];
        ntot += pq.n[k];
    }
    pq.total = sh.total; pq.cnt = w.qcnt; pq.head = w.qhead; pq.err = w.qhead + 32;
    pq.sticky = w.ovf + 1;
    pq.n_blocks = sh.n_blocks;
    pq.spin_limit = sh.spin_limit;
    if (ntot > 0) {
        hipError_t e = queued_variant<T, 0, 2>(c.kappa != 0.0, sh.one_tile, pq, ntot, sh, rho, c, w,
                                               born_R, s, ev, timing_id);
        if (e != hipSuccess) return e;
    }
    const int n_sum = (e_coul || e_gb) ? n_sys : 0;
    const int n_fin = (force || dEdq || dEdrho) ? blocks_for(n_atoms, 256) : 0;
    if (n_sum + n_fin > 0)
        hipLaunchKernelGGL(k_post<T>, dim3(n_sum + n_fin), dim3(256), 0, s, n_atoms, n_sum, w,
                           e_coul, e_gb, dEdq, force, dEdrho, rho, c.offset);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_state_dE(const SiteDev& sd, int n_atoms, const T* x, const T* y, const T* z,
                           const T* q, const GBConst& c, const Work<T>& w, unsigned long long* phi_fx,
                           const int32_t* current_state, const double* pH, const double* E_volt,
                           double T_kelvin, double* dE, double* dG, hipStream_t s, hipEvent_t* ev)
{
    if (sd.n_sites == 0) return hipSuccess;
    if (sd.n_rowitems > 0) {
        hipLaunchKernelGGL(k_clear64, dim3(blocks_for(sd.n_site_atoms, 256)), dim3(256), 0, s, phi_fx,
                           sd.n_site_atoms);
        GBMC_LAUNCH_TIMED(ev, kKSiteRows, k_site_phi_rows<T>, dim3(sd.n_rowitems), dim3(kTile), s,
                          sd.rowitems, sd.site_atoms, w.rows, q, c.kC, c.kT, c.kO, c.kappa, cut2_of(c), phi_fx, w.ovf);
    }
    GBMC_LAUNCH_TIMED(ev, kKSiteDE, k_site_dE<T>, dim3(sd.n_sites), dim3(kSDE), s, sd, x, y, z, q,
                      w.R64, w.A64, c.kC, c.kT, c.kO, c.kappa, cut2_of(c), phi_fx, current_state, pH, E_volt, T_kelvin, dE,
                      dG);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mc_step(const SiteDev& sd, int n_sys, const T* x, const T* y, const T* z,
                          T* q, const GBConst& c, const Work<T>& w, int32_t* current_state,
                          const double* pH, const double* E_volt, double T_kelvin,
                          const double* dE, const double* dG, const double* u,
                          int32_t* n_electrons, int64_t* counters, int32_t* accepted,
                          hipStream_t s, hipEvent_t* ev)
{
    if (n_sys == 0) return hipSuccess;
    GBMC_LAUNCH_TIMED(ev, kKMCStep, k_mc_step<T>, dim3(n_sys), dim3(kMC), s, sd, x, y, z, q, w.R64,
                      w.A64, c.kC, c.kT, c.kO, c.kappa, cut2_of(c), current_state, pH, E_volt, T_kelvin, dE, dG, u, n_electrons,
                      counters, accepted);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mc_sweep(const SiteDev& sd, int n_sys, int n_sa_max, const T* x, const T* y,
                           const T* z, const T* q, T* q_out, const GBConst& c, const Work<T>& w,
                           unsigned long long* phi_fx, int32_t* current_state, const double* pH,
                           const double* E_volt, double T_kelvin, int kinds, const double* u,
                           int32_t* n_electrons, int64_t* counters, int32_t* accepted, double* dG,
                           hipStream_t s)
{
    if (n_sys == 0) return hipSuccess;
    if (sd.n_rowitems > 0) {
        hipLaunchKernelGGL(k_clear64, dim3(blocks_for(sd.n_site_atoms, 256)), dim3(256), 0, s, phi_fx,
                           sd.n_site_atoms);
        hipLaunchKernelGGL(k_site_phi_rows<T>, dim3(sd.n_rowitems), dim3(kTile), 0, s, sd.rowitems,
                           sd.site_atoms, w.rows, q, c.kC, c.kT, c.kO, c.kappa, cut2_of(c), phi_fx, w.ovf);
    }
    const size_t lds = (size_t)6 * sizeof(double) * (size_t)(n_sa_max > 0 ? n_sa_max : 1);
    hipLaunchKernelGGL(k_mc_sweep<T>, dim3(n_sys), dim3(kSweep), lds, s, sd, x, y, z, q, q_out, w.R64,
                       w.A64, c.kC, c.kT, c.kO, c.kappa, cut2_of(c), phi_fx, current_state, pH, E_volt, T_kelvin, kinds, u,
                       n_electrons, counters, accepted, dG);
    return hipGetLastError();
}

hipError_t launch_remd_exchange(int M, const double* E_rung, const int32_t* Ne, int32_t* rep,
                                double T_kelvin, int parity, int wrap, const double* u,
                                int32_t* accepted, double* E_of_rep, hipStream_t s)
{
    if (M < 2) return hipSuccess;
    hipLaunchKernelGGL(k_remd_exchange, dim3(1), dim3(256), 0, s, M, E_rung, Ne, rep, T_kelvin,
                       parity, wrap, u, accepted, E_of_rep);
    return hipGetLastError();
}

#define GBMC_INSTANTIATE(T)                                                                      \
    template hipError_t launch_radii<T>(const WorkItem*, int, int, int, const CutPlan&,         \
                                        const T*,                                                \
                                        const T*, const T*, const T*, const T*, const GBConst&,  \
                                        const Work<T>&, T*, hipStream_t, hipEvent_t*,            \
                                        const T*);                                               \
    template hipError_t launch_energy_forces<T>(const PassShape&, const PassShape&, int, int,      \
                                                const CutPlan&, const T*,                          \
                                                const T*, const T*, const T*, const T*,          \
                                                const T*, const GBConst&, const Work<T>&,        \
                                                double*, double*, T*, T*, T*, hipStream_t,       \
                                                hipEvent_t*, bool);                              \
    template hipError_t launch_queued<T>(const QueueShape&, int, int, const T*, const T*,       \
                                         const T*, const T*, const T*, const T*, const GBConst&, \
                                         const Work<T>&, T*, double*, double*, T*, T*, T*,       \
                                         hipStream_t, hipEvent_t*, int);                         \
    template hipError_t launch_state_dE<T>(const SiteDev&, int, const T*, const T*, const T*,    \
                                           const T*, const GBConst&, const Work<T>&,             \
                                           unsigned long long*,                                  \
                                           const int32_t*, const double*, const double*, double, \
                                           double*, double*, hipStream_t, hipEvent_t*);          \
    template hipError_t launch_mc_step<T>(const SiteDev&, int, const T*, const T*, const T*, T*, \
                                          const GBConst&, const Work<T>&, int32_t*,              \
                                          const double*, const double*, double, const double*,   \
                                          const double*, const double*, int32_t*, int64_t*,      \
                                          int32_t*, hipStream_t, hipEvent_t*);                   \
    template hipError_t launch_mc_sweep<T>(const SiteDev&, int, int, const T*, const T*,          \
                                           const T*, const T*, T*, const GBConst&,               \
                                           const Work<T>&, unsigned long long*, int32_t*,        \
                                           const double*, const double*, double, int,            \
                                           const double*, int32_t*, int64_t*, int32_t*, double*, \
                                           hipStream_t);

GBMC_INSTANTIATE(float)
GBMC_INSTANTIATE(double)

// ====================================================== static scratch
// The workspace of the no-allocation entry point (gb_evaluate_static): one
// library-owned array per GPU, held until the process ends.  In host code the
// name `scratch` is only a host-side stand-in for the symbol; the array's
// device address (one per GPU) is obtained with hipGetSymbolAddress once per
// device, with that device current, and only that address is ever handed to
// kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t scratch_address(int device, void** ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the device must be current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace gbmc
