// The scattering term at discrete angles from the solved modes (Sec. 3.1,
// eq. ani_2d_scattering):  S(x, theta_q) = mu_s sum_{k=-L..L} sigma_hat_|k| u_k(x) e^{i k theta_q},
// theta_q = 2 pi q / ntheta, real part taken.  Pairing k with -k,
//   S = mu_s [ sigma_hat_0 Re u_0 + sum_{k>=1} sigma_hat_k (a_k cos k theta + b_k sin k theta) ]
// with a_k = Re u_k + Re u_{-k} and b_k = Im u_{-k} - Im u_k (channel layout: a_k = sqrt2 c_{2k-1},
// b_k = -sqrt2 c_{2k}).  The work is the output write (8 ntheta bytes per cell against at most
// 16 M bytes read), so one thread keeps one cell's a_k, b_k in registers and writes all of its
// angles; each block builds the cos/sin table of a chunk of angles in LDS, with the angle k q
// reduced exactly modulo ntheta before sincospi.
#include "../../include/rte.h"
#include "ctx.h"

namespace rte {

constexpr int SC_THREADS = 256;
constexpr int SC_QB = 64;   // angles per LDS table chunk

struct ScatterCoef {
    double w[RTE_MAX_L + 1];   // mu_s sigma_hat_k
};

template <int L, bool MODES>
__global__ __launch_bounds__(SC_THREADS) void k_scattering(const double* __restrict__ u, size_t ncell, int ntheta,
                                                           ScatterCoef cf, double* __restrict__ S) {
    __shared__ double2 tab[SC_QB][L > 0 ? L : 1];   // (cos, sin) of k theta_q, k = 1..L
    const size_t i = (size_t)blockIdx.x * SC_THREADS + threadIdx.x;
    const bool live = i < ncell;
    double a0 = 0.0, a[L > 0 ? L : 1], b[L > 0 ? L : 1];
    if (live) {
        if constexpr (MODES) {
            const double2* m = reinterpret_cast<const double2*>(u);
            a0 = cf.w[0] * m[(size_t)L * ncell + i].x;
#pragma unroll
            for (int k = 1; k <= L; ++k) {
                const double2 up = m[(size_t)(L + k) * ncell + i], um = m[(size_t)(L - k) * ncell + i];
                a[k - 1] = cf.w[k] * (up.x + um.x);
                b[k - 1] = cf.w[k] * (um.y - up.y);
            }
        } else {
            const double r2 = 1.4142135623730951;
            a0 = cf.w[0] * u[i];
#pragma unroll
            for (int k = 1; k <= L; ++k) {
                a[k - 1] = cf.w[k] * r2 * u[(size_t)(2 * k - 1) * ncell + i];
                b[k - 1] = -cf.w[k] * r2 * u[(size_t)(2 * k) * ncell + i];
            }
        }
    }
    for (int q0 = 0; q0 < ntheta; q0 += SC_QB) {
        const int nq = min(SC_QB, ntheta - q0);
        if constexpr (L > 0) {
            for (int t = threadIdx.x; t < nq * L; t += SC_THREADS) {
                const int ql = t / L, k = t % L + 1;
                const long long r = ((long long)k * (q0 + ql)) % ntheta;   // exact angle reduction
                double sn, cs;
                sincospi(2.0 * (double)r / (double)ntheta, &sn, &cs);
                tab[ql][k - 1] = make_double2(cs, sn);
            }
            __syncthreads();
        }
        if (live) {
            for (int ql = 0; ql < nq; ++ql) {
                double s = a0;
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    const double2 t = tab[ql][k];
                    s = fma(a[k], t.x, s);
                    s = fma(b[k], t.y, s);
                }
                S[(size_t)(q0 + ql) * ncell + i] = s;
            }
        }
        if constexpr (L > 0) __syncthreads();   // the table is rebuilt for the next chunk
    }
}

template <int L>
static void launch_scatter(const double* u, bool modes, size_t ncell, int ntheta, const ScatterCoef& cf, double* S,
                           hipStream_t st) {
    const unsigned grid = (unsigned)((ncell + SC_THREADS - 1) / SC_THREADS);
    if (modes)
        hipLaunchKernelGGL((k_scattering<L, true>), dim3(grid), dim3(SC_THREADS), 0, st, u, ncell, ntheta, cf, S);
    else
        hipLaunchKernelGGL((k_scattering<L, false>), dim3(grid), dim3(SC_THREADS), 0, st, u, ncell, ntheta, cf, S);
}

}  // namespace rte

using namespace rte;

extern "C" int rte_scattering_term(rte_ctx* c, int layout, const void* u, int ntheta, double* S) {
    if (!c) return set_error(RTE_EINVAL, "ctx is NULL");
    if (layout != RTE_LAYOUT_MODES && layout != RTE_LAYOUT_CHANNELS) return set_error(RTE_EINVAL, "bad layout");
    if (!u || !S) return set_error(RTE_EINVAL, "u or S is NULL");
    if (ntheta < 1 || ntheta > (1 << 24)) return set_error(RTE_EINVAL, "ntheta = %d outside 1..2^24", ntheta);
    if (c->dim != 2) return set_error(RTE_EUNSUPPORTED, "the scattering term at angles is for 2D contexts");
    ScatterCoef cf{};
    for (int k = 0; k <= c->L; ++k) cf.w[k] = c->mu_s * c->sigma[k];
    const bool modes = layout == RTE_LAYOUT_MODES;
    switch (c->L) {
#define RTE_SC_CASE(LL) \
    case LL: launch_scatter<LL>((const double*)u, modes, c->ncell, ntheta, cf, S, c->stream); break;
        RTE_SC_CASE(0) RTE_SC_CASE(1) RTE_SC_CASE(2) RTE_SC_CASE(3) RTE_SC_CASE(4) RTE_SC_CASE(5) RTE_SC_CASE(6)
        RTE_SC_CASE(7) RTE_SC_CASE(8) RTE_SC_CASE(9) RTE_SC_CASE(10) RTE_SC_CASE(11) RTE_SC_CASE(12)
        RTE_SC_CASE(13) RTE_SC_CASE(14) RTE_SC_CASE(15) RTE_SC_CASE(16) RTE_SC_CASE(17) RTE_SC_CASE(18)
        RTE_SC_CASE(19) RTE_SC_CASE(20) RTE_SC_CASE(21) RTE_SC_CASE(22) RTE_SC_CASE(23) RTE_SC_CASE(24)
        RTE_SC_CASE(25) RTE_SC_CASE(26) RTE_SC_CASE(27) RTE_SC_CASE(28) RTE_SC_CASE(29) RTE_SC_CASE(30)
        RTE_SC_CASE(31) RTE_SC_CASE(32)
#undef RTE_SC_CASE
        default: return set_error(RTE_EUNSUPPORTED, "L = %d", c->L);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTE_OK : set_hip_error(e, "rte_scattering_term", __FILE__, __LINE__);
}
