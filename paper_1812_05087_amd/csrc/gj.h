// Dense block inversion in LDS, shared by the block-Jacobi preconditioners.
#pragma once

#include <hip/hip_runtime.h>

namespace fmddm {

constexpr int GJN = 64;  // largest block dimension

// In-place Gauss-Jordan inversion of A[0..nb)[0..nb) (nb <= GJN) by the
// whole workgroup (blockDim.x threads, at least 64), with partial pivoting:
// after step k, column k holds the inverse's column for the row-swapped
// matrix, and the swaps are undone on the columns at the end.  colk and piv
// are LDS scratch of GJN entries.  *bad is set (vector store) when a pivot
// vanishes.
__device__ inline void gj_invert(double (*A)[GJN + 1], int nb, double *colk, int *piv, int *bad)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int k = 0; k < nb; ++k) {
        if (tid < 64) {  // pivot: largest |A[i][k]|, i >= k (smallest i on ties)
            double v = (tid >= k && tid < nb) ? fabs(A[tid][k]) : -1.0;
            int idx = tid;
            for (int o = 32; o > 0; o >>= 1) {
                double v2 = __shfl_xor(v, o);
                int i2 = __shfl_xor(idx, o);
                if (v2 > v || (v2 == v && i2 < idx)) {
                    v = v2;
                    idx = i2;
                }
            }
            if (tid == 0) {
                piv[k] = idx;
                if (!(v > 0.0)) bad[0] = 1;
            }
        }
        __syncthreads();
        int p = piv[k];
        if (p != k)
            for (int j = tid; j < nb; j += nt) {
                double t = A[k][j];
                A[k][j] = A[p][j];
                A[p][j] = t;
            }
        __syncthreads();
        double d = 1.0 / A[k][k];
        if (tid < nb) colk[tid] = A[tid][k];
        __syncthreads();
        // row k scaled, column k replaced, the rest eliminated
        for (int e = tid; e < nb * nb; e += nt) {
            int i = e / nb, j = e % nb;
            if (i == k) A[k][j] = j == k ? d : A[k][j] * d;
            else if (j == k) A[i][k] = -colk[i] * d;
        }
        __syncthreads();
        for (int e = tid; e < nb * nb; e += nt) {
            int i = e / nb, j = e % nb;
            if (i != k && j != k) A[i][j] -= colk[i] * A[k][j];
        }
        __syncthreads();
    }
    for (int k = nb - 1; k >= 0; --k) {
        int p = piv[k];
        if (p != k)
            for (int i = tid; i < nb; i += nt) {
                double t = A[i][k];
                A[i][k] = A[i][p];
                A[i][p] = t;
            }
        __syncthreads();
    }
}

}  // namespace fmddm
