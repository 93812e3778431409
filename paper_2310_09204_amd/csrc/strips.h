// Dense row-strip products on the matrix cores, shared by the matrix-vector product of the solver
// and the block-inverse apply of the preconditioner.
//
// A wave owns 16 consecutive rows of a row-major matrix and a range of columns.  Lane l = 16 kg + i
// streams row i with 16-byte loads at column offset VEC*kg of every 4*VEC-column step, so one
// wave-load covers 16 rows x 4*VEC columns, i.e. VEC slices of the 16x4 A operand of a 16x16x4
// MFMA; the matching B operand X[col][n] comes from the transposed right-hand sides Xt[col][16].
// Operand layout of the 16x16x4 instructions (checked on the device): A[i][k] from lane 16k + i,
// B[k][n] from lane 16k + n; register r of lane l holds D[4(l/16) + r][l%16] for FP32 and
// D[l/16 + 4r][l%16] for FP64.
#pragma once

#include <hip/hip_runtime.h>

namespace bem {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxSplits = 16;

template <typename MT> struct MatrixCore;
template <> struct MatrixCore<float> {
    using V = f32x4;
    static __device__ __forceinline__ int out_row(int kg, int r) { return 4 * kg + r; }
    static __device__ __forceinline__ V mac(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <> struct MatrixCore<double> {
    using V = f64x4;
    static __device__ __forceinline__ int out_row(int kg, int r) { return kg + 4 * r; }
    static __device__ __forceinline__ V mac(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

// acc += rows[16] x Xt over columns [c0, c1) (both multiples of 4*VEC, c1 within the row storage).
// `rowp` points at this lane's row (column 0); rows outside the matrix pass valid = false.
template <typename MT, int UNR>
__device__ __forceinline__ void strip_mfma(const MT* __restrict__ rowp, bool valid, int64_t c0, int64_t c1,
                                           const MT* __restrict__ xt, typename MatrixCore<MT>::V& acc) {
    using MC = MatrixCore<MT>;
    constexpr int VEC = 16 / sizeof(MT);
    constexpr int STEP = 4 * VEC;
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, kg = lane >> 4;
    const MT* w = rowp + VEC * kg;
    const MT* b = xt + int64_t(VEC * kg) * 16 + i;
    for (int64_t jc = c0; jc < c1; jc += STEP * UNR) {
        MT a[UNR][VEC], bx[UNR][VEC];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t col = jc + int64_t(u) * STEP;
            if (col < c1) {
                if (valid) {
                    if constexpr (VEC == 4) {
                        const float4 t = *reinterpret_cast<const float4*>(w + col);
                        a[u][0] = t.x; a[u][1] = t.y; a[u][2] = t.z; a[u][3] = t.w;
                    } else {
                        const double2 t = *reinterpret_cast<const double2*>(w + col);
                        a[u][0] = t.x; a[u][1] = t.y;
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) a[u][v] = MT(0);
                }
#pragma unroll
                for (int v = 0; v < VEC; ++v) bx[u][v] = b[(col + v) * 16];
            } else {
#pragma unroll
                for (int v = 0; v < VEC; ++v) { a[u][v] = MT(0); bx[u][v] = MT(0); }
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc = MC::mac(a[u][v], bx[u][v], acc);
    }
}

}  // namespace bem
