// Real spherical harmonics up to degree 3 as Cartesian polynomials of a unit
// direction (x, y, z), and their gradients.  Basis: from the complex harmonics
// with the Condon-Shortley phase, Y_{l,m>0} = sqrt2 Re Y_l^m,
// Y_{l,0} = Y_l^0, Y_{l,m<0} = sqrt2 Im Y_l^|m|, ordered (l, m) with m
// ascending; on the unit sphere these are the polynomials below, each constant
// being N_l^m times the factor its derivative of P_l contributes.
#pragma once
#include <hip/hip_runtime.h>

namespace cs {

constexpr float SH_C0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float SH_C1 = 0.4886025119029199f;    // sqrt(3/(4 pi))
constexpr float SH_K1 = 1.0925484305920792f;    // sqrt(15/(4 pi))
constexpr float SH_K2 = 0.31539156525252005f;   // sqrt(5/(16 pi))
constexpr float SH_K3 = 0.5462742152960396f;    // sqrt(15/(16 pi))
constexpr float SH_L1 = 0.5900435899266435f;    // sqrt(35/(32 pi))
constexpr float SH_L2 = 2.890611442640554f;     // sqrt(105/(4 pi))
constexpr float SH_L3 = 0.4570457994644658f;    // sqrt(21/(32 pi))
constexpr float SH_L4 = 0.3731763325901154f;    // sqrt(7/(16 pi))
constexpr float SH_L5 = 1.445305721320277f;     // sqrt(105/(16 pi))

// Y[0 .. (deg+1)^2) at unit direction (x, y, z).
__device__ __forceinline__ void sh_eval(int deg, float x, float y, float z, float *Y)
{
    Y[0] = SH_C0;
    if (deg < 1) return;
    Y[1] = -SH_C1 * y;
    Y[2] = SH_C1 * z;
    Y[3] = -SH_C1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = SH_K1 * x * y;
    Y[5] = -SH_K1 * y * z;
    Y[6] = SH_K2 * (3.0f * zz - 1.0f);
    Y[7] = -SH_K1 * x * z;
    Y[8] = SH_K3 * (xx - yy);
    if (deg < 3) return;
    Y[9] = -SH_L1 * y * (3.0f * xx - yy);
    Y[10] = SH_L2 * x * y * z;
    Y[11] = -SH_L3 * y * (5.0f * zz - 1.0f);
    Y[12] = SH_L4 * z * (5.0f * zz - 3.0f);
    Y[13] = -SH_L3 * x * (5.0f * zz - 1.0f);
    Y[14] = SH_L5 * z * (xx - yy);
    Y[15] = -SH_L1 * x * (xx - 3.0f * yy);
}

// g += sum_i w[i] * grad Y_i  (gradient of the polynomials above in R^3).
__device__ __forceinline__ void sh_grad_dot(int deg, float x, float y, float z, const float *w, float &gx, float &gy,
                                            float &gz)
{
    if (deg < 1) return;
    gy += -SH_C1 * w[1];
    gz += SH_C1 * w[2];
    gx += -SH_C1 * w[3];
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    gx += SH_K1 * y * w[4];
    gy += SH_K1 * x * w[4];
    gy += -SH_K1 * z * w[5];
    gz += -SH_K1 * y * w[5];
    gz += 6.0f * SH_K2 * z * w[6];
    gx += -SH_K1 * z * w[7];
    gz += -SH_K1 * x * w[7];
    gx += 2.0f * SH_K3 * x * w[8];
    gy += -2.0f * SH_K3 * y * w[8];
    if (deg < 3) return;
    gx += -6.0f * SH_L1 * x * y * w[9];
    gy += -3.0f * SH_L1 * (xx - yy) * w[9];
    gx += SH_L2 * y * z * w[10];
    gy += SH_L2 * x * z * w[10];
    gz += SH_L2 * x * y * w[10];
    gy += -SH_L3 * (5.0f * zz - 1.0f) * w[11];
    gz += -10.0f * SH_L3 * y * z * w[11];
    gz += SH_L4 * (15.0f * zz - 3.0f) * w[12];
    gx += -SH_L3 * (5.0f * zz - 1.0f) * w[13];
    gz += -10.0f * SH_L3 * x * z * w[13];
    gx += 2.0f * SH_L5 * x * z * w[14];
    gy += -2.0f * SH_L5 * y * z * w[14];
    gz += SH_L5 * (xx - yy) * w[14];
    gx += -3.0f * SH_L1 * (xx - yy) * w[15];
    gy += 6.0f * SH_L1 * x * y * w[15];
}

} // namespace cs
