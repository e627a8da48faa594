// fuse.h - the four fusion rules of Sec. III-C on one channel (device side).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/mem.h"

namespace memk {

// Per-cell coefficients of the Gaussian rule, Eq. (6)-(7), for N
// observations with measurement variance sf2 and prior variance s0
// (+inf = never observed, then the posterior mean is the ML mean).
struct GaussCoef {
    float w0, wa, var;
    bool first;
};

__device__ __forceinline__ GaussCoef gauss_coef(float sf2, float s0, int N)
{
    GaussCoef g;
    float n = (float)N;
    if (isinf(s0)) {
        g.first = true;
        g.w0 = 0.0f;
        g.wa = 1.0f;
        g.var = sf2 / n;
    } else {
        g.first = false;
        float ns0 = n * s0;
        float den = ns0 + sf2;
        g.w0 = sf2 / den;
        g.wa = ns0 / den;
        g.var = (sf2 * s0) / den;
    }
    return g;
}

// New value of one channel under rule R (known at compile time).  a = mean
// of this update's observations (Eq. (1)), sum = their sum, old = stored
// value.
template <int R>
__device__ __forceinline__ float fuse_rule(float param, float old, float a, float sum, const GaussCoef& g)
{
    if constexpr (R == MEM_LATEST)
        return a;
    else if constexpr (R == MEM_EXPAVG)  // Eq. (2); the first observation sets the value
        return isnan(old) ? a : param * a + (1.0f - param) * old;
    else if constexpr (R == MEM_GAUSS)  // Eq. (6)
        return g.first ? a : g.w0 * old + g.wa * a;
    else  // MEM_DIRICHLET, Eq. (12)
        return old + sum;
}

// The same with the rule chosen at run time.
__device__ __forceinline__ float fuse_value(int rule, float param, float old, float a, float sum,
                                            const GaussCoef& g)
{
    switch (rule) {
    case MEM_LATEST: return fuse_rule<MEM_LATEST>(param, old, a, sum, g);
    case MEM_EXPAVG: return fuse_rule<MEM_EXPAVG>(param, old, a, sum, g);
    case MEM_GAUSS: return fuse_rule<MEM_GAUSS>(param, old, a, sum, g);
    default: return fuse_rule<MEM_DIRICHLET>(param, old, a, sum, g);
    }
}

}  // namespace memk
