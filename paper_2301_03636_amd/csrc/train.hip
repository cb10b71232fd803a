// Training of the cost model (section 5.3: the network is fit to measured
// runtimes; here with Adam on the MSE): the forward pass reuses the fused tile
// kernel and saves transposed activations; a fused backward tile kernel runs
// the chain of input gradients through all layers on the matrix cores; split-K
// matrix-core kernels form the weight gradients; loss, gradient norm and the
// order of every reduction are fixed (float64 where the loss and norm are
// summed), so a step is deterministic.
#include <algorithm>
#include <mutex>

#include "mlp_tile.h"

namespace adv {

int repack(advisor_model *m, hipStream_t s);  // model.hip

// ---------------------------------------------------------------------------
// Transposed packed weights for the backward chain: element (k, n) of
// W_l^T (rows = inputs k, reduction over outputs n), same fragment order as
// the forward packing.
template <int P>
__global__ void pack_transposed_kernel(const float *__restrict__ w, int out, int in, int tile_w,
                                       void *__restrict__ dst)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)tile_w * tile_w) return;
    const int k = (int)(idx / tile_w), n = (int)(idx % tile_w);
    const float v = (n < out && k < in) ? w[(int64_t)n * in + k] : 0.0f;
    const int64_t at = pack_index<P>(k, n, tile_w);
    if constexpr (P == PREC_FP32)
        reinterpret_cast<float *>(dst)[at] = v;
    else
        reinterpret_cast<__bf16 *>(dst)[at] = (__bf16)v;
}

template <int P> struct CT;
template <> struct CT<PREC_FP32> { using T = float; };
template <> struct CT<PREC_BF16> { using T = __bf16; };

// ---------------------------------------------------------------------------
// Backward chain over one tile of M rows:
//   g_{L-1}[m][j] = dy[m] * w_out[j] * [h_{L-1}[m][j] > 0]
//   g_{l-1}[m][k] = (sum_n g_l[m][n] W_l[n][k]) * [h_{l-1}[m][k] > 0]
// Each g_l is written transposed ([W][ld], for the weight gradients); the
// chain runs through LDS exactly like the forward pass, with W_l^T packed.
struct BwdArgs {
    const float *dy;        // [n] dL/dyhat
    const float *head_w;    // [W] output-layer weights (padded)
    const void *wt[MAX_LAYERS];
    const void *save_h;     // h_l^T, layer l at l * W * ld
    void *gt;               // g_l^T, layer l at l * W * ld
    float *head_part;       // [ld / M][M / (8 CE)][W + 1] output-layer gradient partials
    const uint32_t *mask;   // ReLU masks of h_0 .. h_{L-2} recorded by the forward
    int64_t ld;
    int64_t n;
    int n_hidden;
};

template <int P, int W, int M, int NWAVES>
__global__ __launch_bounds__(NWAVES * 64) void bwd_tiles_kernel(BwdArgs a)
{
    using C = TileCfg<P, W, M, NWAVES>;
    using G = typename C::G;
    using T = typename CT<P>::T;
    constexpr int CE = 16 / (int)sizeof(T);  // elements per 16-byte run
    constexpr int RG = M / CE;                // row groups of a tile
    static_assert(RG % 8 == 0, "row groups come in eights");
    // the seed pass works in the transposed units of TUnits: UPT units per
    // thread (or one for the first UNITS threads, whole waves), each with
    // all its loads issued before any is used
    using TU = TUnits<P, W, M, C::THREADS>;
    constexpr int UPT = TU::UNITS >= C::THREADS ? TU::UNITS / C::THREADS : 1;
    typedef int v4i_ __attribute__((ext_vector_type(4)));
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char *act = lds;  // [M][AS]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wn = wave % C::WN, wm = wave / C::WN;
    const int nb0 = wn * C::NBW, mb0 = wm * C::MBW;
    const int half = lane >> 5, col = lane & 31;
    const int64_t ld = a.ld, n = a.n;
    const T *H = reinterpret_cast<const T *>(a.save_h);
    T *GT = reinterpret_cast<T *>(a.gt);
    const int L = a.n_hidden;
    const int64_t ntiles = ld / M;

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t row0 = tile * M;
        __syncthreads();
        // seed: gradient at the last hidden layer's pre-activation,
        // g[m][j] = dy[m] w_out[j] [h[m][j] > 0], into LDS (row-major) and out
        // transposed, with the output layer's gradient partials
        // sum_m dy[m] h[m][j] and sum_m dy[m] per line block of rows. dy holds
        // ld rows (those past n are read and then replaced by zero).
        {
            const T *Hl = H + (int64_t)(L - 1) * W * ld;
            T *Gl = GT + (int64_t)(L - 1) * W * ld;
            for (int i = 0; i < UPT; ++i) {
                int c = tid + i * C::THREADS;
                // recompute the unit's addresses here rather than keep them
                // live through the layer loop's multiplies
                asm volatile("" : "+v"(c));
                if (TU::UNITS < C::THREADS && c >= TU::UNITS) break;  // whole waves
                int rg, nq, line;
                TU::decode(c, rg, nq, line);
                v4i_ hraw[2][4], draw[2][CE / 4];
#pragma unroll
                for (int sidx = 0; sidx < 2; ++sidx) {
                    const int64_t r0 = row0 + (rg + 4 * sidx) * CE;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        hraw[sidx][q] = *reinterpret_cast<const v4i_ *>(Hl + (int64_t)(nq * 4 + q) * ld + r0);
#pragma unroll
                    for (int q = 0; q < CE / 4; ++q)
                        draw[sidx][q] = *reinterpret_cast<const v4i_ *>(a.dy + r0 + 4 * q);
                }
                const v4f hw4 = *reinterpret_cast<const v4f *>(a.head_w + nq * 4);
                float sdh[4] = {0.0f, 0.0f, 0.0f, 0.0f}, sd = 0.0f;
#pragma unroll
                for (int sidx = 0; sidx < 2; ++sidx) {
                    const int m0 = (rg + 4 * sidx) * CE;
                    const int64_t r0 = row0 + m0;
                    const float *dv = reinterpret_cast<const float *>(&draw[sidx][0]);
                    v4i_ gvec[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const T *hv = reinterpret_cast<const T *>(&hraw[sidx][q]);
                        T *gv = reinterpret_cast<T *>(&gvec[q]);
#pragma unroll
                        for (int e = 0; e < CE; ++e) {
                            const float d = r0 + e < n ? dv[e] : 0.0f;
                            const float h = (float)hv[e];
                            gv[e] = (T)(h > 0.0f ? d * hw4[q] : 0.0f);
                            sdh[q] += d * h;
                        }
                        *reinterpret_cast<v4i_ *>(Gl + (int64_t)(nq * 4 + q) * ld + r0) = gvec[q];
                    }
#pragma unroll
                    for (int e = 0; e < CE; ++e) sd += r0 + e < n ? dv[e] : 0.0f;
                    lds_scatter4<P>(act, C::AS, m0, nq, gvec);
                }
                // the four lanes of a line block's other row groups; one
                // partial per (tile, line block, neuron), reduced in order by
                // head_reduce_kernel
#pragma unroll
                for (int off = 1; off < 4; off <<= 1) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) sdh[q] += __shfl_xor(sdh[q], off, 64);
                    sd += __shfl_xor(sd, off, 64);
                }
                if ((c & 3) == 0) {
                    float *hp = a.head_part + ((int64_t)tile * (RG / 8) + line) * (W + 1);
                    *reinterpret_cast<v4f *>(hp + nq * 4) = v4f{sdh[0], sdh[1], sdh[2], sdh[3]};
                    if (nq == 0) hp[W] = sd;
                }
            }
        }
        __syncthreads();
        v16f acc[C::NBW][C::MBW];
        for (int l = L - 1; l >= 1; --l) {
            layer_mma<P, W, C::NBW, C::MBW>(reinterpret_cast<const typename G::Vec *>(a.wt[l]),
                                            act, C::AS, nb0, mb0, lane, acc);
            // the ReLU mask of h_{l-1} for this lane's outputs, as the forward
            // recorded it: one word per (32-neuron block, row), this lane's
            // neurons at bits 8 g + 4 half + e
            uint32_t mw[C::NBW][C::MBW];
#pragma unroll
            for (int i = 0; i < C::NBW; ++i)
#pragma unroll
                for (int j = 0; j < C::MBW; ++j)
                    mw[i][j] = a.mask[((int64_t)(l - 1) * (W / 32) + nb0 + i) * ld + row0 +
                                      (mb0 + j) * 32 + col];
            __syncthreads();  // every wave has read g_l
            // g_{l-1} = (sum_n g_l W_l) masked, to LDS for the next layer ...
#pragma unroll
            for (int i = 0; i < C::NBW; ++i)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int kk = (nb0 + i) * 32 + 8 * g + 4 * half;
#pragma unroll
                    for (int j = 0; j < C::MBW; ++j) {
                        const int m = (mb0 + j) * 32 + col;
                        v4f v;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            v[e] = (mw[i][j] >> (8 * g + 4 * half + e)) & 1u ? acc[i][j][4 * g + e] : 0.0f;
                        store4<P>(act + (size_t)m * C::AS, kk, v, 1.0f);
                    }
                }
            __syncthreads();
            // ... and out, transposed, for the weight gradients
            copy_act_transposed<P, W, M, C::THREADS, C::AS>(
                act, GT + (int64_t)(l - 1) * W * ld, ld, row0, n, tid);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient dW[n][k] = sum_b g^T[n][b] h^T[k][b] (both operands with
// the batch contiguous), split over the batch into `splits` ranges whose fp32
// partial tiles are summed in a fixed order by wgrad_reduce_jobs_kernel. A
// workgroup of 4 waves owns a 128 x 128 output tile, each wave 64 x 64.
//
// The batch is consumed in chunks of CH = 8 KV rows (one 128-byte line of
// each operand row). Per chunk the workgroup copies its 128 rows of g^T and
// of h^T into row-padded LDS (eight threads per line, so each line is
// fetched once per workgroup) and every wave reads its fragments from there:
// lane half h takes batch rows h * 4 KV + v * KV + e of its operand row for
// the matrix-core step v = 0..3 (both operands use the same assignment,
// which is all the dot product needs). Two LDS buffers alternate, so the
// copy of the next chunk never waits for the multiplies of this one. The
// waves of the first column tile also sum their g^T rows: the bias
// gradient's partials (one per split, reduced in the same fixed order).
// 72 KB of LDS per workgroup: two workgroups per CU.
//
// One launch holds every layer's product (job j owns workgroups
// [wg0_j, wg0_{j+1}), the last few of each range padding that exit at
// once): a small batch's layers are a few workgroups each, which separate
// launches would run one after another, and a large batch's layers overlap
// each other's first and last waves of workgroups.
struct WgradJob {
    const void *A, *B;       // g^T rows (na of them) and h^T rows (nb), batch-contiguous
    int na, nb, tiles_n, tiles_k, splits, wg0;
    int64_t kchunk;          // batch rows per split
    float *partial, *partial_b, *direct;
    int dout, din;
};
struct WgradJobs {
    int n;
    int64_t ld, n_rows;
    WgradJob job[MAX_LAYERS];
};

template <int P>
__global__ __launch_bounds__(256) void wgrad_kernel(const WgradJobs jobs)
{
    using G = Geo<P>;
    using V = typename G::Vec;
    using T = typename CT<P>::T;
    int jsel = 0;  // the job of this workgroup (uniform)
    for (int q = 1; q < jobs.n; ++q)
        if ((int)blockIdx.x >= jobs.job[q].wg0) jsel = q;
    const WgradJob &J = jobs.job[jsel];
    const T *__restrict__ A = static_cast<const T *>(J.A);
    const T *__restrict__ B = static_cast<const T *>(J.B);
    const int na = J.na, nb = J.nb, tiles_n = J.tiles_n, tiles_k = J.tiles_k, splits = J.splits;
    const int64_t ld = jobs.ld, kchunk = J.kchunk, n_rows = jobs.n_rows;
    float *__restrict__ partial = J.partial;
    float *__restrict__ partial_b = J.partial_b;
    float *__restrict__ direct = J.direct;
    const int dout = J.dout, din = J.din;
    typedef int v4i_ __attribute__((ext_vector_type(4)));
    constexpr int KV = G::KV, CH = 8 * KV;
    constexpr int ROWB = CH * (int)sizeof(T);      // bytes of a row per chunk (128)
    constexpr int SEGS = ROWB / 16;                // 16-byte segments per row (8)
    constexpr int RS = ROWB + 16;                  // padded LDS row stride
    constexpr int TILE = 128 * RS;                 // one operand tile in LDS
    static_assert(SEGS == 8, "a chunk row is one 128-byte line");
    extern __shared__ __align__(16) unsigned char lds[];  // [2][A, B][128][RS]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
    const int half = lane >> 5, col = lane & 31;
    const int wn = wave & 1, wk = wave >> 1;
    // One-dimensional grid of tiles x splits. Workgroups go to the eight
    // XCDs round-robin by id; when the splits divide by 8, XCD x gets splits
    // [x S/8, (x + 1) S/8) for every tile, so each XCD reads its batch range
    // of the operands from HBM once and serves the other tiles' re-reads of
    // the same rows from its own L2.
    int tile, split;
    {
        const int wg = (int)blockIdx.x - J.wg0, tiles = tiles_n * tiles_k;
        if (wg >= tiles * splits) return;  // padding up to the next job's multiple of 8
        if (splits % 8 == 0) {
            const int xcd = wg & 7, slot = wg >> 3;
            split = xcd * (splits >> 3) + slot / tiles;
            tile = slot % tiles;
        } else {
            split = wg / tiles;
            tile = wg % tiles;
        }
    }
    const int n0 = (tile % tiles_n) * 128, k0 = (tile / tiles_n) * 128;
    const int64_t b0 = (int64_t)split * kchunk;
    const bool bias_sums = k0 == 0 && wk == 0;
    bool va[2], vb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        va[i] = n0 + wn * 64 + 32 * i < na;
        vb[i] = k0 + wk * 64 + 32 * i < nb;
    }
    // copy duty: thread covers segment tid % 8 of rows tid / 8 + 32 p, p < 4,
    // of A and of B. Rows past na / nb (whole 32-row groups, never multiplied
    // into a stored output) load row 0 instead, so every load is issued
    // unconditionally and the wait before each copy into LDS can leave the
    // younger chunks' loads in flight.
    const int seg = tid & 7, r0 = tid >> 3;
    const T *pa[4], *pb[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int an = n0 + r0 + 32 * p, bk = k0 + r0 + 32 * p;
        pa[p] = A + (int64_t)(an < na ? an : 0) * ld + b0 + seg * (16 / (int)sizeof(T));
        pb[p] = B + (int64_t)(bk < nb ? bk : 0) * ld + b0 + seg * (16 / (int)sizeof(T));
    }
    auto fetch = [&](int64_t c, v4i_ (&ra)[4], v4i_ (&rb)[4]) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            ra[p] = *reinterpret_cast<const v4i_ *>(pa[p] + c * CH);
            rb[p] = *reinterpret_cast<const v4i_ *>(pb[p] + c * CH);
        }
    };
    auto stash = [&](int buf, const v4i_ (&ra)[4], const v4i_ (&rb)[4]) {
        unsigned char *base = lds + (size_t)buf * 2 * TILE;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int r = r0 + 32 * p;
            *reinterpret_cast<v4i_ *>(base + (size_t)r * RS + seg * 16) = ra[p];
            *reinterpret_cast<v4i_ *>(base + TILE + (size_t)r * RS + seg * 16) = rb[p];
        }
    };
    v16f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v16f{0};
    float rsum[2] = {0.0f, 0.0f};
    // All four products of a wave run even where a 32-row group lies past
    // na or nb: those LDS rows hold copies of row 0 (finite values) and the
    // results are never stored, and one straight-line body keeps the
    // accumulators in place.
    auto compute = [&](int buf) {
        const unsigned char *ab = lds + (size_t)buf * 2 * TILE;
        const unsigned char *bb = ab + TILE;
        V x[4][2];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            V y[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                x[v][i] = *reinterpret_cast<const V *>(ab + (size_t)(wn * 64 + 32 * i + col) * RS + (half * 4 + v) * 16);
                y[i] = *reinterpret_cast<const V *>(bb + (size_t)(wk * 64 + 32 * i + col) * RS + (half * 4 + v) * 16);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if constexpr (P == PREC_FP32) {
#pragma unroll
                        for (int t = 0; t < KV; ++t) acc[i][j] = mma(x[v][i][t], y[j][t], acc[i][j]);
                    } else {
                        acc[i][j] = mma(x[v][i], y[j], acc[i][j]);
                    }
                }
        }
        if (bias_sums) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int e = 0; e < KV; ++e) rsum[i] += (float)x[v][i][e];
        }
    };
    // Three chunks are in flight in registers while one is multiplied out of
    // LDS: stage (c + 1) % 3 holds chunk c + 1 during step c, is copied into
    // the other LDS buffer after the multiplies (its previous contents were
    // last read before the barrier that ended step c - 1), and is refilled
    // with chunk c + 4. The loop runs whole groups of three steps; a step
    // past the last chunk multiplies nothing, and chunk indices past the
    // last load the last chunk again, so every step issues the same loads
    // unconditionally and the compiler's wait before each copy leaves the
    // two younger chunks in flight.
    // chunks of this split's batch range that hold rows (at least one; the
    // rows past n_rows are zero in g^T and add nothing)
    int64_t chunks = kchunk / CH;
    {
        const int64_t live = n_rows - b0;
        if (live < kchunk) chunks = live <= 0 ? 1 : min(chunks, (live + CH - 1) / CH);
    }
    auto clampc = [&](int64_t c) { return c < chunks ? c : chunks - 1; };
    v4i_ sa[3][4], sb[3][4];
    fetch(0, sa[0], sb[0]);
    stash(0, sa[0], sb[0]);
    fetch(clampc(1), sa[1], sb[1]);
    fetch(clampc(2), sa[2], sb[2]);
    fetch(clampc(3), sa[0], sb[0]);
    __syncthreads();
    auto step = [&](int64_t c, v4i_ (&ra)[4], v4i_ (&rb)[4]) {
        if (c < chunks) compute((int)(c & 1));
        stash((int)((c + 1) & 1), ra, rb);
        fetch(clampc(c + 4), ra, rb);
        __syncthreads();
    };
    for (int64_t c = 0; c < chunks; c += 3) {
        step(c, sa[1], sb[1]);
        step(c + 1, sa[2], sb[2]);
        step(c + 2, sa[0], sb[0]);
    }
    // One split (direct != null): the layer's gradient goes straight to its
    // place in the gradient vector, W [dout, din] then the bias, and no
    // reduction follows; otherwise this split's partial tile.
    float *out = partial + (int64_t)split * na * nb;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (!(va[i] && vb[j])) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int nn = n0 + wn * 64 + 32 * i + 8 * (r / 4) + 4 * half + (r % 4);
                const int kk = k0 + wk * 64 + 32 * j + col;
                if (direct) {
                    if (nn < dout && kk < din) direct[(int64_t)nn * din + kk] = acc[i][j][r];
                } else {
                    out[(int64_t)nn * nb + kk] = acc[i][j][r];
                }
            }
        }
    if (bias_sums) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float t = rsum[i] + __shfl_xor(rsum[i], 32, 64);
            const int nn = n0 + wn * 64 + 32 * i + col;
            if (half == 0 && va[i]) {
                if (direct) {
                    if (nn < dout) direct[(int64_t)dout * din + nn] = t;
                } else {
                    partial_b[(int64_t)split * na + nn] = t;
                }
            }
        }
    }
}

constexpr size_t WGRAD_LDS_BYTES = 2 * 2 * 128 * (128 + 16);

// grads[off + n * in + k] = sum over splits of partial[s][n][k] (n < out,
// k < in), then grads[off + out * in + n] = sum over splits of partial_b[s][n]
__device__ __forceinline__ void wgrad_reduce_one(int64_t idx, const float *__restrict__ partial,
                                                 const float *__restrict__ partial_b, int splits,
                                                 int na, int nb, int out, int in,
                                                 float *__restrict__ grads)
{
    const int64_t nw = (int64_t)out * in;
    if (idx >= nw + out) return;
    float s = 0.0f;
    if (idx < nw) {
        const int nn = (int)(idx / in), kk = (int)(idx % in);
        const float *p = partial + (int64_t)nn * nb + kk;
        const int64_t step = (int64_t)na * nb;
#pragma unroll 8
        for (int q = 0; q < splits; ++q) s += p[q * step];
    } else {
        const int nn = (int)(idx - nw);
#pragma unroll 8
        for (int q = 0; q < splits; ++q) s += partial_b[(int64_t)q * na + nn];
    }
    grads[idx] = s;
}

// The same sums four consecutive weights at a time (16-byte loads and
// stores) where the layer's row lengths allow it (in and nb multiples of 4).
__device__ __forceinline__ void wgrad_reduce_four(int64_t idx4, const float *__restrict__ partial,
                                                  const float *__restrict__ partial_b, int splits,
                                                  int na, int nb, int out, int in,
                                                  float *__restrict__ grads)
{
    const int64_t nw4 = (int64_t)out * in / 4;
    if (idx4 < nw4) {
        const int64_t idx = idx4 * 4;
        const int nn = (int)(idx / in), kk = (int)(idx % in);
        const v4f *p = reinterpret_cast<const v4f *>(partial + (int64_t)nn * nb + kk);
        const int64_t step = (int64_t)na * nb / 4;
        v4f s = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 8
        for (int q = 0; q < splits; ++q) {
            const v4f t = p[q * step];
#pragma unroll
            for (int e = 0; e < 4; ++e) s[e] += t[e];
        }
        *reinterpret_cast<v4f *>(grads + idx) = s;
    } else if (idx4 < nw4 + out) {
        const int nn = (int)(idx4 - nw4);
        float s = 0.0f;
#pragma unroll 8
        for (int q = 0; q < splits; ++q) s += partial_b[(int64_t)q * na + nn];
        grads[nw4 * 4 + nn] = s;
    }
}

// The reductions of every layer that split its batch, in one launch: job j
// owns blocks [block0_j, block0_{j+1}) of 256 threads, each thread one output
// (or four consecutive weights when `four`).
struct ReduceJob {
    const float *partial, *partial_b;
    float *grads;
    int splits, na, nb, out, in, four, block0;
};
struct ReduceJobs {
    int n;
    ReduceJob job[MAX_LAYERS];
};

__global__ __launch_bounds__(256) void wgrad_reduce_jobs_kernel(const ReduceJobs jobs)
{
    int jsel = 0;
    for (int q = 1; q < jobs.n; ++q)
        if ((int)blockIdx.x >= jobs.job[q].block0) jsel = q;
    const ReduceJob &J = jobs.job[jsel];
    const int64_t i = (int64_t)((int)blockIdx.x - J.block0) * blockDim.x + threadIdx.x;
    if (J.four)
        wgrad_reduce_four(i, J.partial, J.partial_b, J.splits, J.na, J.nb, J.out, J.in, J.grads);
    else
        wgrad_reduce_one(i, J.partial, J.partial_b, J.splits, J.na, J.nb, J.out, J.in, J.grads);
}

// Output-layer gradient from the backward seed's partials, one workgroup
// per output: for j < in, out[j] = sum over blocks of part[.][j]
// (dW_out = sum_b dy h_{L-1}); out[in] = sum of part[.][W] (db_out =
// sum_b dy). Strided per-thread sums, then a fixed tree: deterministic.
constexpr int HR_THREADS = 256;
__global__ __launch_bounds__(HR_THREADS) void head_reduce_kernel(const float *__restrict__ part,
                                                                 int64_t blocks, int W, int in,
                                                                 float *__restrict__ out)
{
    __shared__ float sh[HR_THREADS];
    const int j = blockIdx.x;
    const int col = j < in ? j : W;
    float s = 0.0f;
    for (int64_t b = threadIdx.x; b < blocks; b += HR_THREADS) s += part[b * (W + 1) + col];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = HR_THREADS / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = sh[0];
}

// ---------------------------------------------------------------------------
// Float64 reductions with a fixed tree: each of RB blocks sums a contiguous
// chunk, then one block sums the RB partials in order.
constexpr int RB = 256, RT = 256;

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = RT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// Loss partials sum (pred - y)^2 and the output gradient dy = 2 (pred - y) / n.
__global__ __launch_bounds__(RT) void loss_kernel(const float *__restrict__ pred,
                                                  const double *__restrict__ y, int64_t n,
                                                  float *__restrict__ dy, double *__restrict__ part)
{
    __shared__ double sh[RT];
    const int64_t chunk = (n + RB - 1) / RB;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += RT) {
        const double r = (double)pred[i] - y[i];
        s += r * r;
        dy[i] = (float)(2.0 * r / (double)n);
    }
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Partials of sum g^2 over the gradient vector.
__global__ __launch_bounds__(RT) void sumsq_kernel(const float *__restrict__ g, int64_t n,
                                                   double *__restrict__ part)
{
    __shared__ double sh[RT];
    const int64_t chunk = (n + RB - 1) / RB;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += RT) {
        const double v = (double)g[i];
        s += v * v;
    }
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Sum of the RB partials by one wave in a fixed order: lane l adds
// part[4l .. 4l+3] in turn, then a butterfly over the lanes (each addition
// pairs the same two values in every lane, so all lanes hold the same,
// run-to-run identical sum). Launched as one workgroup of 64 threads.
static_assert(RB == 4 * 64, "one wave, four partials per lane");
__device__ __forceinline__ double wave_sum_partials(const double *__restrict__ part)
{
    const int l = threadIdx.x & 63;
    double s = part[4 * l];
    s += part[4 * l + 1];
    s += part[4 * l + 2];
    s += part[4 * l + 3];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// out = scale * sum(part[0..RB)), then sqrt if asked.
__global__ void finish_kernel(const double *__restrict__ part, double scale, int take_sqrt,
                              double *__restrict__ out)
{
    double s = wave_sum_partials(part);
    s *= scale;
    if (threadIdx.x == 0) *out = take_sqrt ? sqrt(s) : s;
}

// Adam step counter lives on the device so a captured step replays correctly.
// The same thread forms the step's bias corrections 1 - b^t in float64 once
// (corr[0], corr[1]) for every element of the update to read.
__global__ void step_inc_kernel(int64_t *step, float b1, float b2, double *corr)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t t = *step + 1;
        *step = t;
        corr[0] = 1.0 - pow((double)b1, (double)t);
        corr[1] = 1.0 - pow((double)b2, (double)t);
    }
}

// Adam (Kingma and Ba) on fp32 master weights with the bias corrections of
// the current step (corr, from step_inc_kernel).
__global__ void adam_kernel(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int64_t n, float lr, float b1, float b2,
                            float eps, const double *__restrict__ corr)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float c1 = (float)corr[0];
    const float c2 = (float)corr[1];
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Loss of an RMSprop step from the squared-error partials (the same fixed
// summation order as finish_kernel): the MSE, or for the RMSE loss of
// section 5.3 its square root. The RMSE gradient is the MSE gradient times
// 1 / (2 sqrt(MSE)) (0 when the MSE is 0), so the MSE backward pass serves
// both; scale[0] receives that factor (1 for the MSE loss).
__global__ void loss_scale_kernel(const double *__restrict__ part, double inv_n, int rmse,
                                  double *__restrict__ scale, double *__restrict__ loss_out)
{
    const double mse = wave_sum_partials(part) * inv_n;
    if (threadIdx.x != 0) return;
    const double r = sqrt(mse);
    scale[0] = rmse ? (r > 0.0 ? 0.5 / r : 0.0) : 1.0;
    if (loss_out) *loss_out = rmse ? r : mse;
}

// out = sqrt(sum(part[0..RB))) * scale[0]: the norm of the scaled gradient.
__global__ void scaled_norm_kernel(const double *__restrict__ part,
                                   const double *__restrict__ scale, double *__restrict__ out)
{
    const double s = wave_sum_partials(part);
    if (threadIdx.x == 0) *out = sqrt(s) * scale[0];
}

// RMSprop (section 5.3's optimizer) on fp32 master weights with weight
// decay as an L2 term: g' = c g + wd w, v <- alpha v + (1 - alpha) g'^2,
// w <- w - lr g' / (sqrt(v) + eps), c = scale[0]. With c != 1 the stored
// gradient is replaced by c g, the gradient of the loss being minimized.
__global__ void rmsprop_kernel(float *__restrict__ w, float *__restrict__ v,
                               float *__restrict__ g, int64_t n, float lr, float alpha, float eps,
                               float wd, const double *__restrict__ scale)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double c = *scale;
    float gi = g[i];
    if (c != 1.0) {
        gi = (float)((double)gi * c);
        g[i] = gi;
    }
    const float wi = w[i];
    const float gd = gi + wd * wi;
    const float vi = alpha * v[i] + (1.0f - alpha) * gd * gd;
    v[i] = vi;
    w[i] = wi - lr * gd / (sqrtf(vi) + eps);
}

// ---------------------------------------------------------------------------
// Model-owned training workspace.
struct TrainWs {
    int64_t ld = 0;
    void *saved = nullptr;    // x^T + h_l^T (used by advisor_train_step)
    void *gt = nullptr;       // g_l^T
    float *partial = nullptr; // wgrad partial tiles
    float *head_part = nullptr;  // output-layer gradient partials of the backward seed
    float *pred = nullptr;
    float *dy = nullptr;
    float *grads = nullptr;
    double *red = nullptr;    // 2 x RB partials, then scalars: red[2 RB] loss gradient scale,
                              // red[2 RB + 2 ..] Adam's bias corrections
    void *wt[MAX_LAYERS] = {nullptr};
    size_t partial_floats = 0;
};

static std::mutex g_ws_mu;

static size_t elem_bytes(const advisor_model *m) { return m->precision == PREC_FP32 ? 4 : 2; }

static int64_t ld_for(int64_t n) { return ((n + 255) / 256) * 256; }

// Blocks of output-layer gradient partials the backward seed leaves for a
// batch stride ld: one per 8 row groups of 16 bytes (ld / 64 for bf16,
// ld / 32 for fp32), whatever the tile height.
static int64_t head_blocks(const advisor_model *m, int64_t ld)
{
    return ld / (8 * (16 / (int64_t)elem_bytes(m)));
}

// Batch splits of the weight-gradient product: enough workgroups for two
// per CU (all resident at once, which is what the LDS footprint allows),
// each split a multiple of 64 rows (whole chunks of both precisions).
static int splits_for(int na, int nb, int64_t ld)
{
    const int tiles = ((na + 127) / 128) * ((nb + 127) / 128);
    int s = 1;
    // enough workgroups to fill the device, but at least 512 batch rows per
    // split (a small batch is one split, written without a reduction)
    while (tiles * s < 2 * device_cus() && s < 64 && (int64_t)(2 * s) * 512 <= ld) s *= 2;
    while (s > 1 && (ld / 64) % s != 0) s /= 2;
    return s;
}

// Saved forward state for a batch stride ld: x^T and h_l^T (compute
// precision), then the ReLU mask words of h_0 .. h_{L-2} (one 32-bit word per
// 32-neuron block and row).
static size_t saved_mask_offset(const advisor_model *m, int64_t ld)
{
    return (size_t)(NFEAT + (int64_t)m->n_hidden * m->tile_w) * ld * elem_bytes(m);
}

static size_t saved_bytes_ld(const advisor_model *m, int64_t ld)
{
    const int64_t masked = m->n_hidden > 1 ? m->n_hidden - 1 : 0;
    return saved_mask_offset(m, ld) + (size_t)masked * (m->tile_w / 32) * ld * sizeof(uint32_t);
}

static uint32_t *saved_masks(const advisor_model *m, const void *saved, int64_t ld)
{
    if (m->n_hidden < 2) return nullptr;
    return reinterpret_cast<uint32_t *>(const_cast<unsigned char *>(
        reinterpret_cast<const unsigned char *>(saved) + saved_mask_offset(m, ld)));
}

size_t saved_bytes(const advisor_model *m, int64_t n) { return saved_bytes_ld(m, ld_for(n)); }

TrainWs *train_ws(advisor_model *m) { return reinterpret_cast<TrainWs *>(m->train_ws); }

void free_train_ws(advisor_model *m)
{
    TrainWs *w = train_ws(m);
    if (!w) return;
    void *ptrs[] = {w->saved, w->gt, w->partial, w->pred, w->dy, w->grads, w->red, w->head_part};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (int l = 0; l < MAX_LAYERS; ++l)
        if (w->wt[l]) (void)hipFree(w->wt[l]);
    delete w;
    m->train_ws = nullptr;
}

// Grow the workspace for batches of up to n rows (synchronous allocation).
static int ensure_ws(advisor_model *m, int64_t n, bool with_saved)
{
    TrainWs *w = train_ws(m);
    if (!w) {
        w = new (std::nothrow) TrainWs();
        if (!w) return fail(ADVISOR_ENOMEM, "host allocation");
        m->train_ws = w;
        const int tw = m->tile_w;
        const size_t eb = elem_bytes(m);
        for (int l = 1; l < m->n_hidden; ++l) ADV_HIP(hipMalloc(&w->wt[l], (size_t)tw * tw * eb));
        ADV_HIP(hipMalloc(&w->grads, sizeof(float) * m->n_params));
        ADV_HIP(hipMalloc(&w->red, sizeof(double) * (2 * RB + 8)));  // + scalars
        // every layer's weight partials (all layers' products run in one
        // launch), then every layer's 64 splits x tile width bias partials
        size_t pf = 0;
        for (int l = 0; l < m->n_hidden; ++l) {
            const int na = tw, nb = l == 0 ? NFEAT : tw;
            pf += (size_t)64 * na * nb;
        }
        w->partial_floats = pf;
        ADV_HIP(hipMalloc(&w->partial, sizeof(float) * (pf + (size_t)64 * tw * m->n_hidden)));
    }
    const int64_t ld = ld_for(n);
    if (ld > w->ld || (with_saved && !w->saved)) {
        const int64_t newld = std::max(ld, w->ld);
        for (void **p : {&w->saved, &w->gt, (void **)&w->pred, (void **)&w->dy, (void **)&w->head_part})
            if (*p) { (void)hipFree(*p); *p = nullptr; }
        const size_t eb = elem_bytes(m);
        ADV_HIP(hipMalloc(&w->gt, (size_t)m->n_hidden * m->tile_w * newld * eb));
        ADV_HIP(hipMalloc((void **)&w->head_part,
                          sizeof(float) * (size_t)head_blocks(m, newld) * (m->tile_w + 1)));
        ADV_HIP(hipMalloc((void **)&w->pred, sizeof(float) * newld));
        ADV_HIP(hipMalloc((void **)&w->dy, sizeof(float) * newld));
        ADV_HIP(hipMalloc(&w->saved, saved_bytes_ld(m, newld)));
        w->ld = newld;
    }
    return ADVISOR_OK;
}

// W_l^T packs of layers 1..L-1 from the fp32 master weights.
static int repack_transposed(advisor_model *m, hipStream_t s)
{
    TrainWs *w = train_ws(m);
    const int tw = m->tile_w;
    for (int l = 1; l < m->n_hidden; ++l) {
        const float *src = m->master + m->layer_off[l];
        const unsigned blocks = (unsigned)(((int64_t)tw * tw + 255) / 256);
        if (m->precision == PREC_FP32)
            hipLaunchKernelGGL(pack_transposed_kernel<PREC_FP32>, dim3(blocks), dim3(256), 0, s, src,
                               m->widths[l + 1], m->widths[l], tw, w->wt[l]);
        else
            hipLaunchKernelGGL(pack_transposed_kernel<PREC_BF16>, dim3(blocks), dim3(256), 0, s, src,
                               m->widths[l + 1], m->widths[l], tw, w->wt[l]);
        ADV_LAUNCHED("pack_transposed_kernel");
    }
    m->wt_valid = true;
    return ADVISOR_OK;
}

// After an optimizer step: every compute copy of a trainable (fp32 or bf16)
// model rebuilt from the master parameters in one launch. Jobs are the
// forward packing of each hidden layer, the transposed packing of layers
// 1 .. L-1 and the biases (the same element mappings as pack_layer_kernel,
// pack_transposed_kernel and pack_bias_kernel); the flat index picks the job.
constexpr int PJ_MAX = 2 * ADVISOR_MAX_LAYERS;
struct PackJobs {
    const float *src[PJ_MAX];
    void *dst[PJ_MAX];
    int out[PJ_MAX], in[PJ_MAX], kp[PJ_MAX], transposed[PJ_MAX];
    int64_t start[PJ_MAX + 1];
    int n_jobs;
    int tile_w;
    // biases: hidden layers then the head weights and bias
    const float *master;
    int64_t layer_off[ADVISOR_MAX_LAYERS + 1];
    int widths[ADVISOR_MAX_LAYERS + 1];
    int n_hidden;
    float *bias;
    float *head;
    int64_t total;
};

template <int P>
__global__ void pack_train_kernel(PackJobs a)
{
    using T = typename CT<P>::T;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.total) return;
    if (idx < a.start[a.n_jobs]) {
        int j = 0;
        while (j + 1 < a.n_jobs && idx >= a.start[j + 1]) ++j;
        const int64_t local = idx - a.start[j];
        const int kp = a.kp[j];
        // consecutive threads take consecutive inputs k of one output n, so
        // the master weights are read contiguously; the forward copy puts n
        // in the fragment's rows, the transposed copy puts k there
        const int n = (int)(local / kp), k = (int)(local % kp);
        const float v = (n < a.out[j] && k < a.in[j]) ? a.src[j][(int64_t)n * a.in[j] + k] : 0.0f;
        const int64_t at = a.transposed[j] ? pack_index<P>(k, n, kp) : pack_index<P>(n, k, kp);
        reinterpret_cast<T *>(a.dst[j])[at] = (T)v;
        return;
    }
    const int i = (int)(idx - a.start[a.n_jobs]);
    const int tw = a.tile_w;
    if (i < a.n_hidden * tw) {
        const int l = i / tw, n = i % tw;
        const int in = a.widths[l], out = a.widths[l + 1];
        a.bias[i] = n < out ? a.master[a.layer_off[l] + (int64_t)out * in + n] : 0.0f;
    } else {
        const int j = i - a.n_hidden * tw;
        const int in = a.widths[a.n_hidden];
        const float *hw = a.master + a.layer_off[a.n_hidden];
        a.head[j] = j < tw ? (j < in ? hw[j] : 0.0f) : hw[in];
    }
}

static int repack_train(advisor_model *m, hipStream_t s)
{
    TrainWs *w = train_ws(m);
    PackJobs a{};
    const int tw = m->tile_w;
    int64_t at = 0;
    for (int l = 0; l < m->n_hidden; ++l) {  // forward copies
        const int j = a.n_jobs++;
        a.src[j] = m->master + m->layer_off[l];
        a.dst[j] = m->wpack[l];
        a.out[j] = m->widths[l + 1];
        a.in[j] = m->widths[l];
        a.kp[j] = l == 0 ? NFEAT : tw;
        a.transposed[j] = 0;
        a.start[j] = at;
        at += (int64_t)tw * a.kp[j];
    }
    for (int l = 1; l < m->n_hidden; ++l) {  // transposed copies for the backward chain
        const int j = a.n_jobs++;
        a.src[j] = m->master + m->layer_off[l];
        a.dst[j] = w->wt[l];
        a.out[j] = m->widths[l + 1];
        a.in[j] = m->widths[l];
        a.kp[j] = tw;
        a.transposed[j] = 1;
        a.start[j] = at;
        at += (int64_t)tw * tw;
    }
    a.start[a.n_jobs] = at;
    a.tile_w = tw;
    a.master = m->master;
    for (int l = 0; l <= m->n_hidden; ++l) {
        a.layer_off[l] = m->layer_off[l];
        a.widths[l] = m->widths[l];
    }
    a.widths[m->n_hidden + 1] = m->widths[m->n_hidden + 1];
    a.n_hidden = m->n_hidden;
    a.bias = m->bias;
    a.head = m->head;
    a.total = at + (int64_t)(m->n_hidden + 1) * tw + 1;
    const unsigned blocks = (unsigned)((a.total + 255) / 256);
    if (m->precision == PREC_FP32)
        hipLaunchKernelGGL(pack_train_kernel<PREC_FP32>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(pack_train_kernel<PREC_BF16>, dim3(blocks), dim3(256), 0, s, a);
    ADV_LAUNCHED("pack_train_kernel");
    m->wt_valid = true;
    return ADVISOR_OK;
}

int launch_train_forward(const advisor_model *m, const TileArgs &a, hipStream_t s);  // mlp.hip

template <int P, int W>
struct BwdLaunch {
    static constexpr int M = P == PREC_FP32 ? (W <= 256 ? 128 : (W == 512 ? 64 : 32))
                                            : (W <= 512 ? 128 : 64);
    using C = TileCfg<P, W, M, 8>;
    static constexpr auto kern = bwd_tiles_kernel<P, W, M, 8>;
    static constexpr size_t lds = (size_t)M * C::AS;
    static inline std::once_flag once;
    static inline hipError_t err = hipSuccess;
    static int setup()
    {
        std::call_once(once, [] {
            err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        });
        return err == hipSuccess ? ADVISOR_OK : hip_fail(err, "bwd kernel set-up");
    }
};

template <int P, int W>
static int launch_bwd(const BwdArgs &a, hipStream_t s)
{
    using BL = BwdLaunch<P, W>;
    int rc = BL::setup();
    if (rc) return rc;
    const int64_t ntiles = a.ld / BL::M;
    const int64_t grid = std::min<int64_t>(ntiles, (int64_t)device_cus());
    hipLaunchKernelGGL(BL::kern, dim3((unsigned)grid), dim3(BL::C::THREADS), BL::lds, s, a);
    ADV_LAUNCHED("bwd_tiles_kernel");
    return ADVISOR_OK;
}

// dynamic-LDS limit of the weight-gradient kernels, once per process
static int prepare_wgrad()
{
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        err = hipFuncSetAttribute(reinterpret_cast<const void *>(wgrad_kernel<PREC_FP32>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)WGRAD_LDS_BYTES);
        if (err == hipSuccess)
            err = hipFuncSetAttribute(reinterpret_cast<const void *>(wgrad_kernel<PREC_BF16>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)WGRAD_LDS_BYTES);
    });
    return err == hipSuccess ? ADVISOR_OK : hip_fail(err, "wgrad kernel set-up");
}

int prepare_train_kernels(int precision, int tile_w)
{
    if (int rc = prepare_wgrad()) return rc;
#define ADV_B(P, WW) if (precision == P && tile_w == WW) return BwdLaunch<P, WW>::setup();
    ADV_B(PREC_FP32, 64) ADV_B(PREC_FP32, 128) ADV_B(PREC_FP32, 256) ADV_B(PREC_FP32, 512)
    ADV_B(PREC_FP32, 1024) ADV_B(PREC_BF16, 64) ADV_B(PREC_BF16, 128) ADV_B(PREC_BF16, 256)
    ADV_B(PREC_BF16, 512) ADV_B(PREC_BF16, 1024)
#undef ADV_B
    return fail(ADVISOR_EUNSUPPORTED, "training needs an fp32 or bf16 model");
}

static int dispatch_bwd(const advisor_model *m, const BwdArgs &a, hipStream_t s)
{
#define ADV_B(P, WW) if (m->precision == P && m->tile_w == WW) return launch_bwd<P, WW>(a, s);
    ADV_B(PREC_FP32, 64) ADV_B(PREC_FP32, 128) ADV_B(PREC_FP32, 256) ADV_B(PREC_FP32, 512)
    ADV_B(PREC_FP32, 1024) ADV_B(PREC_BF16, 64) ADV_B(PREC_BF16, 128) ADV_B(PREC_BF16, 256)
    ADV_B(PREC_BF16, 512) ADV_B(PREC_BF16, 1024)
#undef ADV_B
    return fail(ADVISOR_EUNSUPPORTED, "training needs an fp32 or bf16 model");
}

// Gradients of every parameter (fp32, master layout) from the saved forward
// state and dy = dL/dyhat; the core of advisor_mlp_backward and the step.
static int backward_core(advisor_model *m, const float *dy, const void *saved, int64_t n,
                         float *grads, hipStream_t s)
{
    TrainWs *w = train_ws(m);
    const int tw = m->tile_w, L = m->n_hidden;
    const int64_t ld = ld_for(n);
    const size_t eb = elem_bytes(m);
    if (!m->wt_valid) {
        int rc = repack_transposed(m, s);
        if (rc) return rc;
    }
    const unsigned char *xs = reinterpret_cast<const unsigned char *>(saved);
    const unsigned char *hs = xs + (size_t)NFEAT * ld * eb;
    // chain of input gradients through the hidden layers; its seed pass also
    // leaves the partials of the output layer's gradient,
    // dW_out[j] = sum_b dy[b] h_{L-1}[b][j] and db_out = sum_b dy[b]
    BwdArgs a{};
    a.dy = dy;
    a.head_w = m->head;
    a.head_part = w->head_part;
    for (int l = 1; l < L; ++l) a.wt[l] = w->wt[l];
    a.save_h = hs;
    a.mask = saved_masks(m, saved, ld);
    a.gt = w->gt;
    a.ld = ld;
    a.n = n;
    a.n_hidden = L;
    int rc = dispatch_bwd(m, a, s);
    if (rc) return rc;
    {
        float *g_head = grads + m->layer_off[L];
        const int in_last = m->widths[L];
        const int64_t blocks = head_blocks(m, ld);
        hipLaunchKernelGGL(head_reduce_kernel, dim3((unsigned)(in_last + 1)), dim3(HR_THREADS), 0, s,
                           w->head_part, blocks, tw, in_last, g_head);
        ADV_LAUNCHED("head_reduce_kernel");
    }
    // weight and bias gradients per hidden layer
    // one job per layer, all in one launch (each with its own partials, whose
    // splits are then summed per layer in a fixed order); a job's first
    // workgroup is a multiple of 8, so its splits keep their XCD placement
    WgradJobs all{};
    all.ld = ld;
    all.n_rows = n;
    all.n = L;
    size_t pw = 0, pb = 0;
    int wgs = 0;
    for (int l = 0; l < L; ++l) {
        const int na = tw, nb = l == 0 ? NFEAT : tw;
        WgradJob &J = all.job[l];
        J.splits = splits_for(na, nb, ld);
        J.kchunk = ld / J.splits;
        J.A = reinterpret_cast<const unsigned char *>(w->gt) + (size_t)l * tw * ld * eb;
        J.B = l == 0 ? xs : hs + (size_t)(l - 1) * tw * ld * eb;
        J.na = na;
        J.nb = nb;
        J.tiles_n = (na + 127) / 128;
        J.tiles_k = (nb + 127) / 128;
        J.partial = w->partial + pw;
        J.partial_b = w->partial + w->partial_floats + pb;
        pw += (size_t)J.splits * na * nb;
        pb += (size_t)J.splits * na;
        J.wg0 = wgs;
        wgs += (J.tiles_n * J.tiles_k * J.splits + 7) / 8 * 8;
        // weights then biases of the layer (the bias gradient is the sum of
        // g^T's rows over the batch; rows past n are zero)
        J.direct = J.splits == 1 ? grads + m->layer_off[l] : nullptr;
        J.dout = m->widths[l + 1];
        J.din = m->widths[l];
    }
    if (m->precision == PREC_FP32)
        hipLaunchKernelGGL(wgrad_kernel<PREC_FP32>, dim3((unsigned)wgs), dim3(256), WGRAD_LDS_BYTES,
                           s, all);
    else
        hipLaunchKernelGGL(wgrad_kernel<PREC_BF16>, dim3((unsigned)wgs), dim3(256), WGRAD_LDS_BYTES,
                           s, all);
    ADV_LAUNCHED("wgrad_kernel");
    // the split layers' fixed-order reductions, in one launch
    ReduceJobs red{};
    int blocks = 0;
    for (int l = 0; l < L; ++l) {
        const WgradJob &J = all.job[l];
        if (J.direct) continue;
        ReduceJob &R = red.job[red.n++];
        R.partial = J.partial;
        R.partial_b = J.partial_b;
        R.grads = grads + m->layer_off[l];
        R.splits = J.splits;
        R.na = J.na;
        R.nb = J.nb;
        R.out = J.dout;
        R.in = J.din;
        R.four = (R.in % 4 == 0 && R.nb % 4 == 0 && ((uintptr_t)R.grads & 15) == 0) ? 1 : 0;
        const int64_t ne = R.four ? (int64_t)R.out * R.in / 4 + R.out : (int64_t)R.out * R.in + R.out;
        R.block0 = blocks;
        blocks += (int)((ne + 255) / 256);
    }
    if (red.n > 0) {
        hipLaunchKernelGGL(wgrad_reduce_jobs_kernel, dim3((unsigned)blocks), dim3(256), 0, s, red);
        ADV_LAUNCHED("wgrad_reduce_jobs_kernel");
    }
    return ADVISOR_OK;
}

static int check_trainable(const advisor_model *m)
{
    if (!m) return fail(ADVISOR_EINVAL, "null model");
    if (m->precision != PREC_FP32 && m->precision != PREC_BF16)
        return fail(ADVISOR_EUNSUPPORTED, "training needs an fp32 or bf16 model");
    int dev = -1;
    ADV_HIP(hipGetDevice(&dev));
    if (dev != m->device) return fail(ADVISOR_EINVAL, "model lives on another device");
    return ADVISOR_OK;
}

int reserve_train_ws(advisor_model *m, int64_t n)
{
    int rc = check_trainable(m);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_ws_mu);
    return ensure_ws(m, n, true);
}

int repack_transposed_now(advisor_model *m, hipStream_t s)
{
    if (!train_ws(m)) return fail(ADVISOR_EINVAL, "no training workspace");
    return repack_transposed(m, s);
}

}  // namespace adv

using namespace adv;

extern "C" int64_t advisor_mlp_saved_bytes(const advisor_model *m, int64_t n)
{
    if (!m || n < 0) return -1;
    return (int64_t)saved_bytes(m, n);
}

extern "C" int advisor_mlp_forward(advisor_model *m, const int64_t *feat, int64_t n, float *y_out,
                                   void *saved, void *stream)
{
    clear_error();
    int rc = check_trainable(m);
    if (rc) return rc;
    if (n < 1 || n >= ((int64_t)1 << 32)) return fail(ADVISOR_ESHAPE, "row count must be in [1, 2^32)");
    if (!feat || !y_out || !saved) return fail(ADVISOR_EINVAL, "advisor_mlp_forward: null pointer");
    const int64_t ld = ld_for(n);
    TileArgs a{};
    a.feat = feat;
    a.n_rows = n;
    a.pred = y_out;
    a.save_ld = ld;
    a.save_x = saved;
    a.save_h = reinterpret_cast<unsigned char *>(saved) + (size_t)NFEAT * ld * elem_bytes(m);
    a.save_mask = saved_masks(m, saved, ld);
    return launch_train_forward(m, a, as_stream(stream));
}

extern "C" int advisor_mlp_backward(advisor_model *m, const float *dy, const void *saved, int64_t n,
                                    float *grads_out, void *stream)
{
    clear_error();
    int rc = check_trainable(m);
    if (rc) return rc;
    if (n < 1 || n >= ((int64_t)1 << 32)) return fail(ADVISOR_ESHAPE, "row count must be in [1, 2^32)");
    if (!dy || !saved || !grads_out) return fail(ADVISOR_EINVAL, "advisor_mlp_backward: null pointer");
    std::lock_guard<std::mutex> lock(g_ws_mu);
    rc = ensure_ws(m, n, false);
    if (rc) return rc;
    // the backward kernel reads dy in 16-byte vectors over the padded batch:
    // stage the caller's n values in the workspace copy (ld rows)
    TrainWs *w = train_ws(m);
    hipStream_t s = as_stream(stream);
    ADV_HIP(hipMemcpyAsync(w->dy, dy, sizeof(float) * (size_t)n, hipMemcpyDeviceToDevice, s));
    return backward_core(m, w->dy, saved, n, grads_out, s);
}

extern "C" int advisor_train_step(advisor_model *m, const int64_t *feat, const double *y, int64_t n,
                                  float lr, float beta1, float beta2, float eps, double *loss_out,
                                  double *gnorm_out, void *stream)
{
    clear_error();
    int rc = check_trainable(m);
    if (rc) return rc;
    if (n < 1 || n >= ((int64_t)1 << 32)) return fail(ADVISOR_ESHAPE, "row count must be in [1, 2^32)");
    if (!feat || !y) return fail(ADVISOR_EINVAL, "advisor_train_step: null pointer");
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps >= 0.0f))
        return fail(ADVISOR_EINVAL, "bad Adam hyper-parameters");
    std::lock_guard<std::mutex> lock(g_ws_mu);
    rc = ensure_ws(m, n, true);
    if (rc) return rc;
    TrainWs *w = train_ws(m);
    hipStream_t s = as_stream(stream);
    const int64_t ld = ld_for(n);
    // forward, saving what the backward needs
    TileArgs a{};
    a.feat = feat;
    a.n_rows = n;
    a.pred = w->pred;
    a.save_ld = ld;
    a.save_x = w->saved;
    a.save_h = reinterpret_cast<unsigned char *>(w->saved) + (size_t)NFEAT * ld * elem_bytes(m);
    a.save_mask = saved_masks(m, w->saved, ld);
    rc = launch_train_forward(m, a, s);
    if (rc) return rc;
    // float64 MSE and dL/dyhat
    hipLaunchKernelGGL(loss_kernel, dim3(RB), dim3(RT), 0, s, w->pred, y, n, w->dy, w->red);
    if (loss_out)
        hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, w->red, 1.0 / (double)n, 0,
                           loss_out);
    ADV_LAUNCHED("loss kernels");
    rc = backward_core(m, w->dy, w->saved, n, w->grads, s);
    if (rc) return rc;
    // float64 gradient norm
    if (gnorm_out) {
        hipLaunchKernelGGL(sumsq_kernel, dim3(RB), dim3(RT), 0, s, w->grads, m->n_params,
                           w->red + RB);
        hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, w->red + RB, 1.0, 1, gnorm_out);
        ADV_LAUNCHED("gradient norm kernels");
    }
    // Adam on the fp32 master weights, then new compute copies
    double *corr = w->red + 2 * RB + 2;  // workspace scalars: the bias corrections
    hipLaunchKernelGGL(step_inc_kernel, dim3(1), dim3(64), 0, s, m->d_step, beta1, beta2, corr);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((m->n_params + 255) / 256)), dim3(256), 0, s,
                       m->master, m->adam_m, m->adam_v, w->grads, m->n_params, lr, beta1, beta2, eps,
                       (const double *)corr);
    ADV_LAUNCHED("adam_kernel");
    return repack_train(m, s);
}

extern "C" int advisor_train_step_rmsprop(advisor_model *m, const int64_t *feat, const double *y,
                                          int64_t n, float lr, float alpha, float eps,
                                          float weight_decay, int loss, double *loss_out,
                                          double *gnorm_out, void *stream)
{
    clear_error();
    int rc = check_trainable(m);
    if (rc) return rc;
    if (n < 1 || n >= ((int64_t)1 << 32)) return fail(ADVISOR_ESHAPE, "row count must be in [1, 2^32)");
    if (!feat || !y) return fail(ADVISOR_EINVAL, "advisor_train_step_rmsprop: null pointer");
    if (!(lr > 0.0f) || !(alpha >= 0.0f && alpha < 1.0f) || !(eps >= 0.0f) ||
        !(weight_decay >= 0.0f) || !(weight_decay < 1e30f))
        return fail(ADVISOR_EINVAL, "bad RMSprop hyper-parameters");
    if (loss != ADVISOR_LOSS_MSE && loss != ADVISOR_LOSS_RMSE)
        return fail(ADVISOR_EINVAL, "loss must be ADVISOR_LOSS_MSE or ADVISOR_LOSS_RMSE");
    std::lock_guard<std::mutex> lock(g_ws_mu);
    rc = ensure_ws(m, n, true);
    if (rc) return rc;
    TrainWs *w = train_ws(m);
    hipStream_t s = as_stream(stream);
    const int64_t ld = ld_for(n);
    TileArgs a{};
    a.feat = feat;
    a.n_rows = n;
    a.pred = w->pred;
    a.save_ld = ld;
    a.save_x = w->saved;
    a.save_h = reinterpret_cast<unsigned char *>(w->saved) + (size_t)NFEAT * ld * elem_bytes(m);
    a.save_mask = saved_masks(m, w->saved, ld);
    rc = launch_train_forward(m, a, s);
    if (rc) return rc;
    double *scale = w->red + 2 * RB;
    hipLaunchKernelGGL(loss_kernel, dim3(RB), dim3(RT), 0, s, w->pred, y, n, w->dy, w->red);
    hipLaunchKernelGGL(loss_scale_kernel, dim3(1), dim3(64), 0, s, w->red, 1.0 / (double)n,
                       loss == ADVISOR_LOSS_RMSE ? 1 : 0, scale, loss_out);
    ADV_LAUNCHED("loss kernels");
    rc = backward_core(m, w->dy, w->saved, n, w->grads, s);
    if (rc) return rc;
    if (gnorm_out) {
        hipLaunchKernelGGL(sumsq_kernel, dim3(RB), dim3(RT), 0, s, w->grads, m->n_params,
                           w->red + RB);
        hipLaunchKernelGGL(scaled_norm_kernel, dim3(1), dim3(64), 0, s, w->red + RB,
                           (const double *)scale, gnorm_out);
        ADV_LAUNCHED("gradient norm kernels");
    }
    hipLaunchKernelGGL(rmsprop_kernel, dim3((unsigned)((m->n_params + 255) / 256)), dim3(256), 0, s,
                       m->master, m->adam_v, w->grads, m->n_params, lr, alpha, eps, weight_decay,
                       (const double *)scale);
    ADV_LAUNCHED("rmsprop_kernel");
    return repack_train(m, s);
}

// Section 5.3's learning rate: lr0 for the first `every` epochs, then
// multiplied by gamma after each further `every` epochs.
extern "C" double advisor_step_lr(int64_t epoch, double lr0, double gamma, int64_t every)
{
    clear_error();
    if (epoch < 0 || every < 1 || !(lr0 > 0.0) || !(gamma > 0.0 && gamma <= 1.0)) {
        fail(ADVISOR_EINVAL, "advisor_step_lr: need epoch >= 0, every >= 1, lr0 > 0, 0 < gamma <= 1");
        return __builtin_nan("");
    }
    return lr0 * pow(gamma, (double)(epoch / every));
}

// Replace the fp32 master parameters from a device buffer (for optimizers
// driven outside the library) and rebuild every compute copy.
extern "C" int advisor_model_load_params(advisor_model *m, const float *w_master, void *stream)
{
    clear_error();
    if (!m || !w_master) return fail(ADVISOR_EINVAL, "load_params: null pointer");
    if (m->precision == PREC_FP8)
        return fail(ADVISOR_EUNSUPPORTED, "fp8 models take parameters through set_params");
    hipStream_t s = as_stream(stream);
    ADV_HIP(hipMemcpyAsync(m->master, w_master, sizeof(float) * m->n_params,
                           hipMemcpyDeviceToDevice, s));
    int rc = repack(m, s);
    if (rc) return rc;
    m->wt_valid = false;
    return ADVISOR_OK;
}

extern "C" int advisor_model_grads(const advisor_model *m, float *grads_out, void *stream)
{
    clear_error();
    if (!m || !grads_out) return fail(ADVISOR_EINVAL, "model_grads: null pointer");
    TrainWs *w = reinterpret_cast<TrainWs *>(m->train_ws);
    if (!w) return fail(ADVISOR_EINVAL, "no training step has run on this model");
    ADV_HIP(hipMemcpyAsync(grads_out, w->grads, sizeof(float) * m->n_params,
                           hipMemcpyDeviceToDevice, as_stream(stream)));
    return ADVISOR_OK;
}
