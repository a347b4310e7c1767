// Forward kinematics of the robot on the device (Section 3.2: the action
// offsets are applied to the state, then the link frames follow).
#pragma once

#include "gal_internal.h"
#include "gal_math.h"

namespace gal {

// The eight frames of pose `st` (10 floats): link 0 = base, links 1..7 =
// the DH joint frames, each the product of its predecessor with
// A_j = Rz(q_j) Tz(d_j) Tx(a_j) Rx(alpha_j).
struct Fk {
    Frame f[8];
};

__device__ __forceinline__ void forward_kinematics(const RobotParams &rp, const float *st, Fk &out)
{
    float s, c;
    dsincos(st[2], s, c);
    Frame F0;
    F0.m[0] = c;    F0.m[1] = -s;   F0.m[2] = 0.0f;  F0.m[3] = st[0];
    F0.m[4] = s;    F0.m[5] = c;    F0.m[6] = 0.0f;  F0.m[7] = st[1];
    F0.m[8] = 0.0f; F0.m[9] = 0.0f; F0.m[10] = 1.0f; F0.m[11] = 0.0f;
    Frame T;
    T.m[0] = 1.0f; T.m[1] = 0.0f; T.m[2] = 0.0f;  T.m[3] = rp.mount[0];
    T.m[4] = 0.0f; T.m[5] = 1.0f; T.m[6] = 0.0f;  T.m[7] = rp.mount[1];
    T.m[8] = 0.0f; T.m[9] = 0.0f; T.m[10] = 1.0f; T.m[11] = rp.mount[2];
    out.f[0] = F0;
    Frame prev = fmul(F0, T);
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        float sq, cq;
        dsincos(st[3 + j], sq, cq);
        const float a = rp.dh[j][0], d = rp.dh[j][1], ca = rp.dh[j][2], sa = rp.dh[j][3];
        Frame A;
        A.m[0] = cq;   A.m[1] = -(sq * ca); A.m[2] = sq * sa;     A.m[3] = a * cq;
        A.m[4] = sq;   A.m[5] = cq * ca;    A.m[6] = -(cq * sa);  A.m[7] = a * sq;
        A.m[8] = 0.0f; A.m[9] = sa;         A.m[10] = ca;         A.m[11] = d;
        prev = fmul(prev, A);
        out.f[j + 1] = prev;
    }
}

}  // namespace gal
