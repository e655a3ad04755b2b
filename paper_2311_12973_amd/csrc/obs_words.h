// obs_words.h — a run's observations as the 32-bit words the filter kernel reads.
//
// Epidemic models observe counts: one int32 per observed series and day (four series
// for the age-structured model). The linear-Gaussian model observes one FP64 value a
// day, staged as its two 32-bit halves, low word first.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/smc2.h"

namespace smc2 {

inline int obs_words(int model)
{
    if (model == SMC2_AGE_SEIR) return 4;
    if (model == SMC2_LINGAUSS) return 2;
    return 1;
}

// nullptr when the run's observations are valid for the model, else the reason
inline const char* obs_check(int model, const smc2_run& r)
{
    if (model == SMC2_LINGAUSS) {
        if (!r.y_real) return "null observations (y_real)";
        for (int t = 0; t < r.T; ++t)
            if (!std::isfinite(r.y_real[t])) return "non-finite observation";
        return nullptr;
    }
    if (!r.y) return "null observations";
    const int no = obs_words(model);
    for (int e = 0; e < r.T * no; ++e)
        if (r.y[e] < 0) return "negative observation";
    return nullptr;
}

// Appends the run's T x obs_words(model) words to out.
inline void obs_pack(int model, const smc2_run& r, std::vector<int32_t>& out)
{
    if (model == SMC2_LINGAUSS) {
        for (int t = 0; t < r.T; ++t) {
            uint64_t b;
            std::memcpy(&b, r.y_real + t, sizeof(b));
            out.push_back((int32_t)(uint32_t)b);
            out.push_back((int32_t)(uint32_t)(b >> 32));
        }
        return;
    }
    out.insert(out.end(), r.y, r.y + (size_t)r.T * obs_words(model));
}

}  // namespace smc2
