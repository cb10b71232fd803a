// Variant generation (section 4.1.3): for every kernel with n collapsible
// loops (1 <= n <= 4), the placements of the parallel-for directive (merged
// with teams distribute at loop 0 with collapse 1..n; or at loop x, 1 <= x <
// n, with teams distribute collapsing 1..x loops and parallel for 1..n-x),
// times the allowed schedules, times the two data-transfer options:
// n^3 + 5n variants per kernel with all three schedules. Integer work only:
// a count pass with a prefix sum gives the offsets, then each kernel's rows
// are written by one wave, every lane decoding the rows of the words it
// stores so the stores are contiguous.
#include <algorithm>

#include "internal.h"

namespace adv {

namespace {

constexpr int VG_THREADS = 256;
constexpr int VG_ITEMS = 4;                        // kernels per thread in the scan
constexpr int VG_BLOCK = VG_THREADS * VG_ITEMS;    // kernels per scan block
constexpr int VG_WAVES = VG_THREADS / 64;

// placements of the parallel-for directive for n loops: n + sum x (n - x)
__device__ __forceinline__ int64_t vg_placements(int64_t n)
{
    if (n < 1 || n > ADVISOR_MAX_LOOPS) return 0;
    int64_t p = n;
    for (int64_t x = 1; x < n; ++x) p += x * (n - x);
    return p;
}

__device__ __forceinline__ int64_t vg_count(int64_t n, int n_sched)
{
    return vg_placements(n) * n_sched * 2;
}

// exclusive prefix sum over the block's threads (LDS, Hillis-Steele)
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *sh, int64_t *total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < VG_THREADS; off <<= 1) {
        const int64_t add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const int64_t incl = sh[t];
    *total = sh[VG_THREADS - 1];
    __syncthreads();
    return incl - v;
}

// per-block sums of the variant counts
__global__ __launch_bounds__(VG_THREADS) void vg_block_sums_kernel(
    const int64_t *__restrict__ n_loops, int64_t n_k, int n_sched, int64_t *__restrict__ sums)
{
    __shared__ int64_t sh[VG_THREADS];
    const int64_t base = (int64_t)blockIdx.x * VG_BLOCK + (int64_t)threadIdx.x * VG_ITEMS;
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < VG_ITEMS; ++j)
        if (base + j < n_k) s += vg_count(n_loops[base + j], n_sched);
    int64_t total;
    (void)block_exclusive_scan(s, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive scan of the block sums in place, one workgroup, in chunks
__global__ __launch_bounds__(VG_THREADS) void vg_scan_sums_kernel(int64_t *__restrict__ sums,
                                                                 int64_t n_blocks)
{
    __shared__ int64_t sh[VG_THREADS];
    int64_t carry = 0;
    for (int64_t base = 0; base < n_blocks; base += VG_THREADS) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < n_blocks ? sums[i] : 0;
        int64_t total;
        const int64_t ex = block_exclusive_scan(v, sh, &total);
        if (i < n_blocks) sums[i] = carry + ex;
        carry += total;
    }
}

// offsets[k] = start of kernel k's rows; the last block also writes offsets[n_k]
__global__ __launch_bounds__(VG_THREADS) void vg_offsets_kernel(
    const int64_t *__restrict__ n_loops, int64_t n_k, int n_sched,
    const int64_t *__restrict__ sums, int64_t *__restrict__ offsets)
{
    __shared__ int64_t sh[VG_THREADS];
    const int64_t base = (int64_t)blockIdx.x * VG_BLOCK + (int64_t)threadIdx.x * VG_ITEMS;
    int64_t c[VG_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < VG_ITEMS; ++j) {
        c[j] = base + j < n_k ? vg_count(n_loops[base + j], n_sched) : 0;
        s += c[j];
    }
    int64_t total;
    int64_t run = sums[blockIdx.x] + block_exclusive_scan(s, sh, &total);
#pragma unroll
    for (int j = 0; j < VG_ITEMS; ++j) {
        if (base + j < n_k) offsets[base + j] = run;
        run += c[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == VG_THREADS - 1) offsets[n_k] = run;
}

__global__ void vg_zero_kernel(int64_t *p) { *p = 0; }

// One wave per kernel: the segment's words [6 off[k], 6 off[k+1]), clamped to
// the output, written in order; the word's row r (local index) decodes as
// data = r mod 2, schedule = the (r / 2 mod n_sched)-th allowed schedule,
// placement = r / (2 n_sched) in the order x = 0 (c = 1..n), then x = 1..n-1
// with (d, c) row-major over 1..x by 1..n-x. Rows past the kernel's own
// count (offsets not from the count pass) are written as -1.
//
// The decode depends only on (n, r) and the schedule mask, so each workgroup
// first decodes every row of every loop count (VG_TABLE entries) into LDS,
// four bits per field; a row then costs one LDS read. Each lane writes
// whole rows (48 bytes: three 16-byte stores where the output is 16-byte
// aligned, so the wave's three stores fill 3 KB of the output together). A
// wave takes VG_KPW consecutive kernels at a time: their offsets and loop
// counts come in one load, one per lane, so a wave pays one memory round
// trip for several kernels' rows.
constexpr int VG_KPW = 8;

__device__ __forceinline__ int64_t read_lane_i64(int64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
constexpr int VG_TABLE = 6 + 18 + 42 + 84;  // n^3 + 5n rows for n = 1..4

__device__ __forceinline__ int vg_table_base(int n)  // first entry of loop count n
{
    return n == 1 ? 0 : (n == 2 ? 6 : (n == 3 ? 24 : 66));
}

__global__ __launch_bounds__(VG_THREADS) void vg_rows_kernel(
    const int64_t *__restrict__ n_loops, const int64_t *__restrict__ offsets, int64_t n_k,
    int64_t n_v, int sched_mask, int n_sched, int64_t *__restrict__ out)
{
    static_assert(ADVISOR_VARIANT_COLS == 6 && ADVISOR_MAX_LOOPS == 4, "table layout");
    __shared__ uint32_t table[VG_TABLE];
    for (int t = threadIdx.x; t < VG_TABLE; t += VG_THREADS) {
        const int nn = t < 6 ? 1 : (t < 24 ? 2 : (t < 66 ? 3 : 4));
        const int r = t - vg_table_base(nn);
        uint32_t e = 0xffffffffu;  // rows past this mask's count: never read
        if (r < vg_count(nn, n_sched)) {
            const int data = r & 1;
            const int q = r >> 1;
            const int si = q % n_sched;
            int p = q / n_sched;
            int sch = 0;
            for (int b = 0, seen = 0; b < 3; ++b)
                if ((sched_mask >> b) & 1) {
                    if (seen == si) sch = b;
                    ++seen;
                }
            int x = 0, d = 0, c = 0;
            if (p < nn) {
                c = p + 1;
            } else {
                p -= nn;
                for (x = 1; x < nn; ++x) {
                    const int m = x * (nn - x);
                    if (p < m) break;
                    p -= m;
                }
                d = p / (nn - x) + 1;
                c = p % (nn - x) + 1;
            }
            e = (uint32_t)x | ((uint32_t)d << 4) | ((uint32_t)c << 8) | ((uint32_t)sch << 12) |
                ((uint32_t)data << 16);
        }
        table[t] = e;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * VG_WAVES;
    const bool wide = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
    typedef long long v2ll_ __attribute__((ext_vector_type(2)));
    const int64_t wave0 = (int64_t)blockIdx.x * VG_WAVES + (threadIdx.x >> 6);
    for (int64_t k0 = wave0 * VG_KPW; k0 < n_k; k0 += nwaves * VG_KPW) {
        // lane j holds offsets[k0 + j] (j <= VG_KPW) and n_loops[k0 + j]
        const int64_t kl = k0 + lane;
        const int64_t offl = lane <= VG_KPW && kl <= n_k ? offsets[kl] : 0;
        const int64_t nl = lane < VG_KPW && kl < n_k ? n_loops[kl] : 0;
        const int nb = (int)min((int64_t)VG_KPW, n_k - k0);
        for (int j = 0; j < nb; ++j) {
            const int64_t k = k0 + j;
            const int64_t seg0 = read_lane_i64(offl, j);
            const int64_t lo = max((int64_t)0, min(seg0, n_v));
            const int64_t hi = max(lo, min(read_lane_i64(offl, j + 1), n_v));
            const int64_t n = read_lane_i64(nl, j);
            const int64_t cnt = vg_count(n, n_sched);
            const int base = cnt > 0 ? vg_table_base((int)n) : 0;
            for (int64_t row = lo + lane; row < hi; row += 64) {
                const int64_t r64 = row - seg0;
                int64_t v[ADVISOR_VARIANT_COLS] = {-1, -1, -1, -1, -1, -1};
                if (r64 >= 0 && r64 < cnt) {
                    // at most 84 rows per kernel: a 32-bit index into the table
                    const uint32_t e = table[base + (int)r64];
                    v[0] = k;
#pragma unroll
                    for (int c = 1; c < ADVISOR_VARIANT_COLS; ++c) v[c] = (int64_t)((e >> (4 * (c - 1))) & 15u);
                }
                int64_t *o = out + row * ADVISOR_VARIANT_COLS;
                if (wide) {
#pragma unroll
                    for (int c = 0; c < ADVISOR_VARIANT_COLS; c += 2)
                        *reinterpret_cast<v2ll_ *>(o + c) = v2ll_{v[c], v[c + 1]};
                } else {
#pragma unroll
                    for (int c = 0; c < ADVISOR_VARIANT_COLS; ++c) o[c] = v[c];
                }
            }
        }
    }
}

int check_variant_args(const int64_t *n_loops, int64_t n_k, int sched_mask)
{
    if (sched_mask < 1 || sched_mask > 7) return fail(ADVISOR_EINVAL, "sched_mask must be in [1, 7]");
    if (n_k < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_k >= (int64_t)1 << 31) return fail(ADVISOR_ESHAPE, "n_kernels must be < 2^31");
    if (n_k > 0 && !n_loops) return fail(ADVISOR_EINVAL, "null n_loops");
    return ADVISOR_OK;
}

// A generated variant as a cost-model descriptor row (one thread per row):
// [k, x, d, c, s, data] -> [k, c + 8 x + 64 d + 512 s, teams, threads, maps],
// the maps being the kernel's analysed classes (data option 0) or tofrom for
// every array (option 1), 0 past the kernel's arrays. A row whose kernel id
// is out of range keeps that id (the featurizer marks it invalid).
__global__ __launch_bounds__(VG_THREADS) void vg_lower_kernel(
    const int64_t *__restrict__ kdesc, const int64_t *__restrict__ gen, int64_t n_k, int64_t n_v,
    int64_t teams, int64_t threads, int64_t *__restrict__ vdesc)
{
    const int64_t i = (int64_t)blockIdx.x * VG_THREADS + threadIdx.x;
    if (i >= n_v) return;
    const int64_t *g = gen + i * ADVISOR_VARIANT_COLS;
    const int64_t k = g[0], x = g[1], d = g[2], c = g[3], sch = g[4], data = g[5];
    longlong2 r0, r1, r2, r3;
    r0.x = k;
    r0.y = c + 8 * x + 64 * d + 512 * sch;
    r1.x = teams;
    r1.y = threads;
    int64_t m[4] = {0, 0, 0, 0};
    if (k >= 0 && k < n_k) {
        const int64_t *kd = kdesc + k * KD;
        const int64_t A = kd[5];
#pragma unroll
        for (int a = 0; a < 4; ++a) m[a] = a < A ? (data == 0 ? kd[12 + a] : 3) : 0;
    }
    r2.x = m[0];
    r2.y = m[1];
    r3.x = m[2];
    r3.y = m[3];
    longlong2 *out = reinterpret_cast<longlong2 *>(vdesc + i * VD);
    out[0] = r0;
    out[1] = r1;
    out[2] = r2;
    out[3] = r3;
}

}  // namespace

}  // namespace adv

using namespace adv;

extern "C" int advisor_lower_variants(const int64_t *kdesc, const int64_t *variants,
                                      int64_t n_kernels, int64_t n_variants, int64_t teams,
                                      int64_t threads, int64_t *vdesc_out, void *stream)
{
    clear_error();
    if (n_kernels < 0 || n_variants < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_variants >= (int64_t)1 << 32) return fail(ADVISOR_ESHAPE, "n_variants must be < 2^32");
    if (teams < 1 || threads < 1) return fail(ADVISOR_EINVAL, "teams and threads must be >= 1");
    if (n_variants == 0) return ADVISOR_OK;
    if (!variants || !vdesc_out || (n_kernels > 0 && !kdesc))
        return fail(ADVISOR_EINVAL, "advisor_lower_variants: null pointer");
    const int64_t blocks = (n_variants + VG_THREADS - 1) / VG_THREADS;
    hipLaunchKernelGGL(vg_lower_kernel, dim3((unsigned)blocks), dim3(VG_THREADS), 0,
                       as_stream(stream), kdesc, variants, n_kernels, n_variants, teams, threads,
                       vdesc_out);
    ADV_LAUNCHED("vg_lower_kernel");
    return ADVISOR_OK;
}

extern "C" int advisor_count_variants(const int64_t *n_loops, int64_t n_kernels, int sched_mask,
                                      int64_t *offsets_out, void *stream)
{
    clear_error();
    if (int rc = check_variant_args(n_loops, n_kernels, sched_mask)) return rc;
    if (!offsets_out) return fail(ADVISOR_EINVAL, "null offsets_out");
    hipStream_t s = as_stream(stream);
    if (n_kernels == 0) {
        hipLaunchKernelGGL(vg_zero_kernel, dim3(1), dim3(1), 0, s, offsets_out);
        ADV_LAUNCHED("vg_zero_kernel");
        return ADVISOR_OK;
    }
    const int n_sched = __builtin_popcount((unsigned)sched_mask);
    const int64_t n_blocks = (n_kernels + VG_BLOCK - 1) / VG_BLOCK;
    int64_t *sums = nullptr;
    ADV_HIP(hipMallocAsync((void **)&sums, sizeof(int64_t) * n_blocks, s));
    hipLaunchKernelGGL(vg_block_sums_kernel, dim3((unsigned)n_blocks), dim3(VG_THREADS), 0, s,
                       n_loops, n_kernels, n_sched, sums);
    hipLaunchKernelGGL(vg_scan_sums_kernel, dim3(1), dim3(VG_THREADS), 0, s, sums, n_blocks);
    hipLaunchKernelGGL(vg_offsets_kernel, dim3((unsigned)n_blocks), dim3(VG_THREADS), 0, s,
                       n_loops, n_kernels, n_sched, (const int64_t *)sums, offsets_out);
    hipError_t le = hipGetLastError();
    hipError_t fe = hipFreeAsync(sums, s);
    if (le != hipSuccess) return hip_fail(le, "variant count kernels");
    if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync");
    return ADVISOR_OK;
}

extern "C" int advisor_enumerate_variants(const int64_t *n_loops, const int64_t *offsets,
                                          int64_t n_kernels, int64_t n_variants, int sched_mask,
                                          int64_t *variants_out, void *stream)
{
    clear_error();
    if (int rc = check_variant_args(n_loops, n_kernels, sched_mask)) return rc;
    if (n_variants < 0) return fail(ADVISOR_ESHAPE, "negative size");
    if (n_variants >= ((int64_t)1 << 62) / ADVISOR_VARIANT_COLS)
        return fail(ADVISOR_ESHAPE, "n_variants too large");
    if (n_kernels == 0 || n_variants == 0) return ADVISOR_OK;
    if (!offsets || !variants_out) return fail(ADVISOR_EINVAL, "advisor_enumerate_variants: null pointer");
    hipStream_t s = as_stream(stream);
    const int n_sched = __builtin_popcount((unsigned)sched_mask);
    const int64_t blocks =
        std::min<int64_t>((n_kernels + VG_WAVES * VG_KPW - 1) / (VG_WAVES * VG_KPW), 1 << 20);
    hipLaunchKernelGGL(vg_rows_kernel, dim3((unsigned)blocks), dim3(VG_THREADS), 0, s, n_loops,
                       offsets, n_kernels, n_variants, sched_mask, n_sched, variants_out);
    ADV_LAUNCHED("vg_rows_kernel");
    return ADVISOR_OK;
}
