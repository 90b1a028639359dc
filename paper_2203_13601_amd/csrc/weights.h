// Weight settings of the fusion distance (Eq. 6).  The default (w_v = 1,
// w_l = delta / m, Sec. 3.2) orders by the square-root-free key
// delta^2 (m_q + chi)^2.  The other settings of the sensitivity study
// (Sec. 6.5, Fig. 10 (i); Eq. 8) order by Gamma itself, evaluated with one
// rounding per operation and no fused multiply-add, in float32 for the
// search and the candidate tiles and in float64 for the build's exact keys.
#pragma once

#include <cstdint>

#include "nhq.h"

namespace nhq {

struct Weights {
    int mode;   // NHQ_WEIGHTS_*
    float p;    // c (Eq. 8), delta_max or the ratio w_l / w_v
    double pd;  // the same parameter as the caller gave it
};

// Gamma for a pair at vector distance delta with chi mismatches out of m_q
// constrained attributes (m_q = m between two objects)
__device__ __forceinline__ float w_gamma32(float delta, int chi, int mq, const Weights &w)
{
#pragma clang fp contract(off)
    float c = (float)chi;
    switch (w.mode) {
    case NHQ_WEIGHTS_HARMONIC: {
        const float u = delta + c;
        if (u == 0.0f)
            return 0.0f;
        return (2.0f * delta * c) / u;
    }
    case NHQ_WEIGHTS_HARMONIC_C:
        c = chi == 0 ? 1.0f : w.p * c;
        return (2.0f * delta * c) / (delta + c);
    case NHQ_WEIGHTS_NORMALISED:
        return delta / w.p + (mq == 0 ? 0.0f : c / (float)mq);
    case NHQ_WEIGHTS_FIXED:
        return delta + w.p * c;
    default:
        return mq == 0 ? delta : delta * ((float)(mq + chi) / (float)mq);
    }
}

// ordering key from delta^2 (float32)
__device__ __forceinline__ float w_key32(float d2, int chi, int mq, const Weights &w)
{
    if (w.mode == NHQ_WEIGHTS_DEFAULT)
        return mq == 0 ? d2 : d2 * (float)((mq + chi) * (mq + chi));
    return w_gamma32(__builtin_sqrtf(d2), chi, mq, w);
}

// ordering key from delta^2 (float64, the build's exact re-score)
__device__ __forceinline__ double w_key64(double d2, int chi, int mq, const Weights &w)
{
#pragma clang fp contract(off)
    if (w.mode == NHQ_WEIGHTS_DEFAULT)
        return mq == 0 ? d2 : d2 * (double)((mq + chi) * (mq + chi));
    const double delta = __builtin_sqrt(d2);
    double c = (double)chi;
    switch (w.mode) {
    case NHQ_WEIGHTS_HARMONIC:
        return (delta + c == 0.0) ? 0.0 : (2.0 * delta * c) / (delta + c);
    case NHQ_WEIGHTS_HARMONIC_C:
        c = chi == 0 ? 1.0 : w.pd * c;
        return (2.0 * delta * c) / (delta + c);
    case NHQ_WEIGHTS_NORMALISED:
        return delta / w.pd + (mq == 0 ? 0.0 : c / (double)mq);
    default:  // NHQ_WEIGHTS_FIXED
        return delta + w.pd * c;
    }
}

}  // namespace nhq
