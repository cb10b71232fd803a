// Device-side feature extraction of one variant (one thread per variant).
//
// The kernel facts come from the kernel analysis of section 4.1 (loop nest,
// arrays, data classes of section 4.1.2) and the variant's choices from the
// variant generation of section 4.1.3 (collapse, teams, threads, map). The
// paper feeds 33 unlisted features to its network (section 5.3); the 32
// defined here are documented in include/advisor.h next to
// advisor_featurize. Unsigned 64-bit arithmetic throughout (modulo 2^64).
#pragma once

#include "internal.h"

namespace adv {

// Map clause m carries the data an array of class req needs: alloc needs
// nothing, to needs to/tofrom, from needs from/tofrom, tofrom needs tofrom.
// A 4x4 bit table indexed by (req, m).
__device__ __forceinline__ bool map_ok(int64_t req, int64_t m)
{
    if ((uint64_t)req > 3u || (uint64_t)m > 3u) return false;
    constexpr uint32_t table = 0xFu | (0xAu << 4) | (0xCu << 8) | (0x8u << 12);
    return (table >> (req * 4 + m)) & 1u;
}

struct Feat {
    uint64_t f[NFEAT];
};

// Reads the variant row v (8 int64) and, if its kernel id is in range, the
// kernel row. Returns false and zeroes the features for an invalid variant.
// Column 1 is the parallel structure c + 8 x + 64 d + 512 s of section 4.1.3
// (parallel for at loop x with collapse c, teams-distribute collapse d,
// schedule s): x = 0 is the combined directive over loops 0 .. c-1; at
// x >= 1 the teams share loops 0 .. d-1 and each team's threads loops
// x .. x+c-1, the loops between and after running serially.
__device__ __forceinline__ bool featurize_one(const int64_t *__restrict__ kdesc,
                                              const int64_t *__restrict__ vrow, int64_t n_k,
                                              Feat &out)
{
#pragma unroll
    for (int j = 0; j < NFEAT; ++j) out.f[j] = 0;
    const longlong2 *v2 = reinterpret_cast<const longlong2 *>(vrow);
    longlong2 va = v2[0], vb = v2[1], vc = v2[2], vd = v2[3];
    const int64_t kid = va.x, cf = va.y, T = vb.x, H = vb.y;
    const int64_t c = cf & 7, x = (cf >> 3) & 7, d = (cf >> 6) & 7, sch = cf >> 9;
    const int64_t m[4] = {vc.x, vc.y, vd.x, vd.y};
    if (kid < 0 || kid >= n_k) return false;
    const longlong2 *k2 = reinterpret_cast<const longlong2 *>(kdesc + kid * KD);
    int64_t k[KD];
#pragma unroll
    for (int q = 0; q < KD / 2; ++q) {
        longlong2 t = k2[q];
        k[2 * q] = t.x;
        k[2 * q + 1] = t.y;
    }
    const int64_t D = k[0], A = k[5], E = k[6], fpi = k[11];
    bool ok = D >= 1 && D <= 4 && A >= 0 && A <= 4 && E >= 1 && E <= 64 && fpi >= 0 &&
              T >= 1 && H >= 1 && cf >= 0 && sch <= 2 && c >= 1 &&
              (x == 0 ? (d == 0 && c <= D) : (x < D && d >= 1 && d <= x && c <= D - x));
#pragma unroll
    for (int i = 0; i < 4; ++i) ok = ok && k[1 + i] >= 1 && (i < D || k[1 + i] == 1);
#pragma unroll
    for (int a = 0; a < 4; ++a)
        ok = ok && (a >= A || ((uint64_t)k[7 + a] <= 1u && map_ok(k[12 + a], m[a])));
    if (!ok) return false;

    const uint64_t N0 = k[1], N1 = k[2], N2 = k[3], N3 = k[4];
    const uint64_t I = N0 * N1 * N2 * N3;
    const uint64_t TH = (uint64_t)T * (uint64_t)H;
    uint64_t Pc, R, busy, waves, npar;
    if (x == 0) {
        // collapsed loops 0..c-1 form the parallel space, the rest run serially
        Pc = N0;
        R = N1 * N2 * N3;
        if (c >= 2) { Pc *= N1; R = N2 * N3; }
        if (c >= 3) { Pc *= N2; R = N3; }
        if (c >= 4) { Pc *= N3; R = 1; }
        busy = TH < Pc ? TH : Pc;
        const uint64_t q = Pc / TH;
        waves = q + (Pc - q * TH != 0);
        npar = c;
    } else {
        // teams over loops 0..d-1, a team's threads over loops x..x+c-1
        const uint64_t Nv[4] = {N0, N1, N2, N3};
        uint64_t Pt = 1, Pf = 1;
        R = 1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool team = i < d, thr = i >= x && i < x + c;
            Pt *= team ? Nv[i] : 1;
            Pf *= thr ? Nv[i] : 1;
            R *= (team || thr) ? 1 : Nv[i];
        }
        Pc = Pt * Pf;
        const uint64_t T64 = (uint64_t)T, H64 = (uint64_t)H;
        busy = (T64 < Pt ? T64 : Pt) * (H64 < Pf ? H64 : Pf);
        const uint64_t qt = Pt / T64, qf = Pf / H64;
        waves = (qt + (Pt - qt * T64 != 0)) * (qf + (Pf - qf * H64 != 0));
        npar = d + c;
    }
    const uint64_t S = (uint64_t)E * I;
    // arrays per map clause and strided arrays (no indexed register arrays)
    uint64_t c_alloc = 0, c_to = 0, c_from = 0, c_tofrom = 0, ns = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (a < A) {
            c_alloc += m[a] == 0;
            c_to += m[a] == 1;
            c_from += m[a] == 2;
            c_tofrom += m[a] == 3;
            ns += (uint64_t)k[7 + a];
        }
    }
    const uint64_t cnt[4] = {c_alloc, c_to, c_from, c_tofrom};
    const uint64_t h2d = S * (cnt[1] + cnt[3]);
    const uint64_t d2h = S * (cnt[2] + cnt[3]);
    const uint64_t line = (uint64_t)(64u / (uint32_t)E);
    uint64_t *f = out.f;
    f[0] = D;
    f[1] = N0; f[2] = N1; f[3] = N2; f[4] = N3;
    f[5] = I;
    f[6] = npar;
    f[7] = Pc;
    f[8] = R;
    f[9] = T;
    f[10] = H;
    f[11] = TH;
    f[12] = busy;
    f[13] = waves;
    f[14] = waves * R;
    f[15] = waves * TH - Pc;
    f[16] = A;
    f[17] = E;
    f[18] = S;
    f[19] = cnt[1];
    f[20] = cnt[2];
    f[21] = cnt[3];
    f[22] = cnt[0];
    f[23] = h2d;
    f[24] = d2h;
    f[25] = h2d + d2h;
    f[26] = ns;
    f[27] = S * (uint64_t)A;
    f[28] = S * ((uint64_t)A - ns) + line * S * ns;
    f[29] = (uint64_t)fpi * I;
    f[30] = fpi;
    f[31] = S * cnt[0];
    return true;
}

// Z-score of one integer feature in float64: (log2(1 + f) - mu) / sigma.
__device__ __forceinline__ double zscore(int64_t f, double mu, double sigma)
{
    return (log2((double)f + 1.0) - mu) / sigma;
}

// The same standardization as the network's float32 input, at a fraction of
// the cost. 1 + f is formed in float64 and split as m * 2^e with m in
// [1/2, 1); the exponent enters exactly and only log2(m), in [-1, 0), is taken
// in float32 with the hardware base-2 logarithm (about one ulp there), so the
// logarithm's absolute error stays near 1e-7 whatever the feature's
// magnitude. The centred value goes to float32 before the reciprocal scale.
// f = -1 gives -inf and f < -1 NaN, as the float64 definition does.
__device__ __forceinline__ float zscore_fast(int64_t f, double mu, double sigma)
{
    int e;
    const double m = frexp((double)f + 1.0, &e);
    const double l = (double)e + (double)__builtin_amdgcn_logf((float)m);
    return (float)(l - mu) * __builtin_amdgcn_rcpf((float)sigma);
}

}  // namespace adv
