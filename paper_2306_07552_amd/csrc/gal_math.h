// Device arithmetic of the step, as fixed sequences of binary32 operations
// (each rounds once to nearest-even; kernels are built with
// -ffp-contract=off so no multiply-add is fused).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gal {

// sin and cos by Cody-Waite reduction modulo pi/2 (pi/2 split into an
// 8-significant-bit head and a tail, so k*head is exact for small k) followed
// by Taylor polynomials of degree 9 (sin) and 8 (cos) on [-pi/4, pi/4], whose
// truncation error is below half an ulp of 1.  Quadrant from k mod 4.
__device__ __forceinline__ void dsincos(float x, float &s, float &c)
{
    const float two_over_pi = 0x1.45f306p-1f;
    const float pio2_hi = 0x1.92p+0f;
    const float pio2_lo = 0x1.fb5444p-12f;
    float k = rintf(x * two_over_pi);
    float r = (x - k * pio2_hi) - k * pio2_lo;
    float r2 = r * r;
    // 1/9!, -1/7!, 1/5!, -1/3! and 1/8!, -1/6!, 1/4!, -1/2! rounded to float
    float ps = ((0x1.71de3ap-19f * r2 + -0x1.a01a02p-13f) * r2 + 0x1.111112p-7f) * r2
               + -0x1.555556p-3f;
    float pc = ((0x1.a01a02p-16f * r2 + -0x1.6c16c2p-10f) * r2 + 0x1.555556p-5f) * r2 + -0.5f;
    float sr = r + (r * r2) * ps;
    float cr = 1.0f + r2 * pc;
    int q = ((int)k) & 3;
    float ss = (q & 1) ? cr : sr;
    float cc = (q & 1) ? sr : cr;
    // quadrant signs: q=0 (+s,+c) 1 (+c,-s) 2 (-s,-c) 3 (-c,+s)
    s = (q == 2 || q == 3) ? -ss : ss;
    c = (q == 1 || q == 2) ? -cc : cc;
}

// 3x4 rigid transforms, row-major (R | t).  Products accumulate left to
// right: ((a0*b0 + a1*b1) + a2*b2), translation added last.
struct Frame {
    float m[12];
};

__device__ __forceinline__ Frame fmul(const Frame &A, const Frame &B)
{
    Frame C;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float t = A.m[i * 4 + 0] * B.m[j] + A.m[i * 4 + 1] * B.m[4 + j];
            C.m[i * 4 + j] = t + A.m[i * 4 + 2] * B.m[8 + j];
        }
        float t = A.m[i * 4 + 0] * B.m[3] + A.m[i * 4 + 1] * B.m[7];
        t = t + A.m[i * 4 + 2] * B.m[11];
        C.m[i * 4 + 3] = t + A.m[i * 4 + 3];
    }
    return C;
}

__device__ __forceinline__ void fpoint(const Frame &F, float px, float py, float pz,
                                       float &ox, float &oy, float &oz)
{
    ox = ((F.m[0] * px + F.m[1] * py) + F.m[2] * pz) + F.m[3];
    oy = ((F.m[4] * px + F.m[5] * py) + F.m[6] * pz) + F.m[7];
    oz = ((F.m[8] * px + F.m[9] * py) + F.m[10] * pz) + F.m[11];
}

__device__ __forceinline__ void fvec(const Frame &F, float vx, float vy, float vz,
                                     float &ox, float &oy, float &oz)
{
    ox = (F.m[0] * vx + F.m[1] * vy) + F.m[2] * vz;
    oy = (F.m[4] * vx + F.m[5] * vy) + F.m[6] * vz;
    oz = (F.m[8] * vx + F.m[9] * vy) + F.m[10] * vz;
}

}  // namespace gal
