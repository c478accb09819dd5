// Host-side interface of the 3D isotropic apply passes B, C, D (A and E are the 2D x-passes).
#pragma once
#include "common.h"

namespace rte {

template <typename T>
struct Apply3DArgs {
    int nx, ny, nz, PX, PY, PZ;
    cx<T>* T1;                 // [nz][PX/2+1][ny]
    cx<T>* T2;                 // [PX/2+1][PY][nz]
    const T* Q3;               // [PX/2+1][PY/2+1][PZ/2+1], scaled by 1/(PX PY PZ)
    const cx<T>* twy;
    const cx<T>* twz;
    hipStream_t stream;
};

// which = 1: y-FFT with transposed store; 2: z-FFT, spectrum multiply, inverse z-FFT;
// 3: inverse y-FFT back to T1.
template <typename T>
int apply3d_pass(const Apply3DArgs<T>& a, int which);

}  // namespace rte
