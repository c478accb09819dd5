// Real spherical harmonics of the 3D anisotropic modes (Sec. 3.1.2), host and device.
//
// Mode a = l^2 + l + m (l = 0..L, m = -l..l) is the real harmonic, normalised to unit mean square
// over the sphere:
//     Y_{l,0}   = sqrt(2l+1) q_l^0(z)
//     Y_{l,+-m} = sqrt(2 (2l+1) (l-m)!/(l+m)!) q_l^m(z) {Re, Im} (x + i y)^m      (m > 0)
// on the unit vector (x, y, z), where q_l^m(z) = P_l^m(z) / (1 - z^2)^(m/2) is the associated
// Legendre function without the Condon-Shortley phase and without its sine power (which
// (x + i y)^m carries), by the recurrences q_m^m = (2m - 1)!!, q_{m+1}^m = (2m + 1) z q_m^m,
// (l - m) q_l^m = (2l - 1) z q_{l-1}^m - (l + m - 1) q_{l-2}^m.
// So Y_00 = 1, (Y_{1,-1}, Y_{1,0}, Y_{1,1}) = sqrt(3) (y, z, x).
//
// Parities under reflection of one axis (used to keep one octant of every kernel spectrum):
//   y -> -y: +1 for m >= 0, -1 for m < 0;   z -> -z: (-1)^(l - |m|).
#pragma once
#include <cmath>

#include "common.h"

namespace rte {

constexpr int sh_modes(int L) { return (L + 1) * (L + 1); }
__host__ __device__ constexpr int sh_degree(int a) {
    int l = 0;
    while ((l + 1) * (l + 1) <= a) ++l;
    return l;
}
__host__ __device__ constexpr int sh_order(int a) { return a - sh_degree(a) * sh_degree(a) - sh_degree(a); }
__host__ __device__ constexpr int sh_parity_y(int a) { return sh_order(a) < 0 ? -1 : 1; }
__host__ __device__ constexpr int sh_parity_z(int a) {
    return ((sh_degree(a) - (sh_order(a) < 0 ? -sh_order(a) : sh_order(a))) & 1) ? -1 : 1;
}

__host__ __device__ inline double real_sh_lm(int l, int m, double x, double y, double z) {
    const int am = m < 0 ? -m : m;
    double cr = 1.0, ci = 0.0;                  // (x + i y)^|m|
    for (int k = 0; k < am; ++k) {
        const double t = cr * x - ci * y;
        ci = cr * y + ci * x;
        cr = t;
    }
    double q = 1.0;                             // q_{|m|}^{|m|} = (2|m| - 1)!!
    for (int k = 1; k <= am; ++k) q *= 2.0 * k - 1.0;
    if (l > am) {
        double qm1 = q, qc = (2.0 * am + 1.0) * z * q;
        for (int ll = am + 2; ll <= l; ++ll) {
            const double qn = ((2.0 * ll - 1.0) * z * qc - (ll + am - 1.0) * qm1) / (ll - am);
            qm1 = qc;
            qc = qn;
        }
        q = qc;
    }
    double ratio = 1.0;                         // (l - |m|)! / (l + |m|)!
    for (int k = l - am + 1; k <= l + am; ++k) ratio /= (double)k;
    const double nrm = sqrt((am == 0 ? 1.0 : 2.0) * (2.0 * l + 1.0) * ratio);
    return nrm * q * (m > 0 ? cr : (m < 0 ? ci : 1.0));
}

__host__ __device__ inline double real_sh(int a, double x, double y, double z) {
    return real_sh_lm(sh_degree(a), sh_order(a), x, y, z);
}

}  // namespace rte
