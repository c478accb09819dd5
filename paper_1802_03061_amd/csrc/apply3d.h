// Host-side interface of the 3D apply passes B, C, D (A and E are the 2D x-passes).
#pragma once
#include "common.h"

namespace rte {

// Per-channel factor applied when pass B loads a channel (the diagonal D of the operator).
struct ChanScale3 {
    double s[16];
};

template <typename T>
struct Apply3DArgs {
    int nx, ny, nz, PX, PY, PZ;
    int C;                     // channels: 1 (isotropic) or (L+1)^2 spherical-harmonic modes
    int L;
    cx<T>* T1;                 // [C][nz][PX/2+1][ny]
    cx<T>* T2;                 // [C][PX/2+1][PY][nz]
    const T* Q3;               // isotropic: octant [PX/2+1][PY/2+1][PZ/2+1], scaled by 1/(PX PY PZ);
                               // C > 1: one such octant per mode pair a <= b (spectra.h)
    const cx<T>* twy;
    const cx<T>* twz;
    ChanScale3 sc;             // factor per channel on the pass-B load
    hipStream_t stream;
    int var[3] = {0, 0, 0};    // kernel variants of passes B, C, D (apply3d_variant_count)
};

// Kernel variants of the 3D passes B, C, D (which = 1, 2, 3), same arithmetic, different tiling:
// B and D take 8, 4 or 16 z-rows per block; the isotropic C takes 2048/PZ, half or twice as many
// columns per block; the spherical-harmonic C has one form.
template <typename T>
int apply3d_variant_count(int which, int C, int PZ);

// which = 1: y-FFT with transposed store; 2: z-FFT, spectrum multiply (C > 1: the mode coupling),
// inverse z-FFT; 3: inverse y-FFT back to T1.
template <typename T>
int apply3d_pass(const Apply3DArgs<T>& a, int which);

}  // namespace rte
