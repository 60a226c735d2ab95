// Complex arithmetic of the complex-parameter RBM kernels (FP32).
#pragma once

#include <hip/hip_runtime.h>

namespace nqs {

__device__ inline float2 cmul(float2 x, float2 y) { return make_float2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x); }

// tanh(x + iy) = (sinh 2x + i sin 2y) / (cosh 2x + cos 2y)
__device__ inline float2 ctanh(float2 z)
{
    const float ax = fminf(fabsf(2.0f * z.x), 80.0f);
    const float e = __expf(ax), ei = 1.0f / e;
    const float ch = 0.5f * (e + ei), sh = copysignf(0.5f * (e - ei), z.x);
    float sy, cy;
    sincosf(2.0f * z.y, &sy, &cy);
    const float den = ch + cy;
    return make_float2(sh / den, sy / den);
}

// log |cosh(x + iy)| = 0.5 log((cosh 2x + cos 2y) / 2)
__device__ inline float clogcosh_re(float2 z)
{
    const float ax = fabsf(2.0f * z.x);
    // cosh 2x + cos 2y = e^{|2x|} (1 + e^{-2|2x|}) / 2 + cos 2y
    const float e = __expf(-ax);
    const float v = 0.5f * (1.0f + e * e) + cosf(2.0f * z.y) * e;
    return 0.5f * (ax + logf(v)) - 0.5f * 0.6931471805599453f;
}

}  // namespace nqs
