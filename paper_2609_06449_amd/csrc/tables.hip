// Host-side twiddle tables shared by the single-transform plan (plan.hip)
// and the batched plan (batch.hip).  Every entry is exp(-2 pi i r / M) for an
// exactly reduced integer r, evaluated in FP64 and rounded once to FP32, so
// two plans of the same transform size hold bit-identical tables.
#include <cmath>

#include "paco_internal.h"

namespace paco {

float2 root_neg(int64_t r, int64_t M)
{
    const double a = 2.0 * M_PI * (double(r) / double(M));
    return make_float2(float(std::cos(a)), float(-std::sin(a)));
}

bool stage_tables(std::vector<float2> &stw, int64_t off[kMaxOnChipLog2 + 1])
{
    stw.clear();
    off[0] = 0;
    for (int l = 1; l <= kMaxOnChipLog2; ++l) {
        off[l] = int64_t(stw.size());
        for (int S = 1; S < stage_count(l); ++S) {
            const int R = 1 << stage_log2radix(l, S);
            const int64_t Ns = int64_t(1) << stage_log2ns(l, S), M = Ns * R;
            const int LOW = stage_lo_width(l, S), HIW = stage_hi_width(l, S);
            for (int r = 1; r < R; ++r)
                for (int kl = 0; kl < LOW; ++kl) stw.push_back(root_neg((int64_t(kl) * r) % M, M));
            for (int r = 1; r < R; ++r)
                for (int kh = 0; kh < HIW; ++kh) stw.push_back(root_neg((int64_t(16) * kh * r) % M, M));
        }
        if (int64_t(stw.size()) - off[l] != stage_tw_total(l)) return false;
    }
    stw.push_back(make_float2(0.f, 0.f));  // never empty
    return true;
}

void middle_tables(int lN, std::vector<float2> &hi, std::vector<float2> &lo, std::vector<float2> &tile)
{
    const int64_t N = int64_t(1) << lN;
    const int lLo = middle_log2lo(lN);
    const int64_t Lo = int64_t(1) << lLo, Hi = N >> lLo;
    constexpr int64_t TT = kTwTile;
    hi.resize(Hi);
    lo.resize(Lo);
    tile.resize(TT * TT);
    for (int64_t h = 0; h < Hi; ++h) hi[h] = root_neg(h * Lo, N);
    for (int64_t l = 0; l < Lo; ++l) lo[l] = root_neg(l, N);
    for (int64_t i = 0; i < TT; ++i)
        for (int64_t j = 0; j < TT; ++j) tile[i * TT + j] = root_neg((i * j) % N, N);
}

}  // namespace paco
