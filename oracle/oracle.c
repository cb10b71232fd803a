/*
 * CPU oracle for the cost-model hot path of the OpenMP Advisor paper
 * (arXiv 2301.03636): featurize -> Z-score -> MLP -> per-kernel argmin,
 * plus the MSE loss, its gradient and the Adam update used to train it.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library. The product path
 * never links or calls it, and it shares no code, header or table with the
 * HIP library.
 *
 * Plain C, float64 throughout, loops in the order the definitions give, no
 * blocking, no fusion, no BLAS. Integer work uses unsigned 64-bit arithmetic
 * (wrapping modulo 2^64, so every input has a defined result; in the
 * documented domain nothing wraps and the values are the exact integers).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KD_COLS 16
#define VD_COLS 8
#define NFEAT 32

enum { CLS_ALLOC = 0, CLS_TO = 1, CLS_FROM = 2, CLS_TOFROM = 3 };

/* Is map clause m allowed for an array whose data class is req?  Section
 * 4.1.2 classifies every array as alloc / to / from / tofrom: a "to" array
 * must reach the device, a "from" array must come back, a "tofrom" array
 * both ways, an "alloc" array needs neither. A clause is allowed when it moves
 * at least that data. */
static int map_allowed(int64_t req, int64_t m)
{
    if (req < 0 || req > 3 || m < 0 || m > 3) return 0;
    switch (req) {
    case CLS_ALLOC: return 1;
    case CLS_TO: return m == CLS_TO || m == CLS_TOFROM;
    case CLS_FROM: return m == CLS_FROM || m == CLS_TOFROM;
    default: return m == CLS_TOFROM;
    }
}

/*
 * Feature extraction (the "Feature Extraction" box of the training and
 * prediction flows, section 3; 33 features in section 5.3, never listed in
 * the paper). The 32 int64 features of one variant, from the kernel facts
 * the kernel analysis records (section 4.1: loop nest, arrays, data classes)
 * and the variant's choices (section 4.1.3: collapse, teams, threads, map).
 * Returns 1 if the variant is valid, 0 (and a zero row) if it is not.
 *
 * The variant's parallel structure (column 1) is c + 8 x + 64 d + 512 s, the
 * parameters of section 4.1.3: the parallel-for directive at loop x with
 * collapse c, a teams-distribute collapse d, and the schedule s (0 static,
 * 1 dynamic, 2 guided). At x = 0 the two directives are one combined
 * directive over loops 0 .. c-1 (d = 0, 1 <= c <= D): its Pc iterations are
 * spread over all T x H threads. At 1 <= x < D, teams distribute loops
 * 0 .. d-1 (1 <= d <= x; Pt iterations over the T teams) and each team's H
 * threads share loops x .. x+c-1 (1 <= c <= D - x; Pf iterations); the loops
 * between (d .. x-1) and after (x+c ..) run serially.
 */
static int featurize_row(const int64_t *kd, const int64_t *vd, int64_t n_k, int64_t *f)
{
    memset(f, 0, sizeof(int64_t) * NFEAT);
    int64_t kid = vd[0];
    if (kid < 0 || kid >= n_k) return 0;
    kd += kid * KD_COLS;
    int64_t D = kd[0], A = kd[5], E = kd[6], fpi = kd[11];
    int64_t cf = vd[1], T = vd[2], H = vd[3];
    if (cf < 0 || cf >= 1536) return 0;
    int64_t c = cf % 8, x = (cf / 8) % 8, d = (cf / 64) % 8, sched = cf / 512;
    if (D < 1 || D > 4) return 0;
    for (int i = 0; i < 4; i++) {
        if (kd[1 + i] < 1) return 0;
        if (i >= D && kd[1 + i] != 1) return 0;
    }
    if (A < 0 || A > 4 || E < 1 || E > 64 || fpi < 0) return 0;
    if (T < 1 || H < 1 || sched > 2) return 0;
    if (x == 0 && (d != 0 || c < 1 || c > D)) return 0;
    if (x >= 1 && (x >= D || d < 1 || d > x || c < 1 || c > D - x)) return 0;
    for (int a = 0; a < A; a++) {
        if (kd[7 + a] < 0 || kd[7 + a] > 1) return 0;
        if (!map_allowed(kd[12 + a], vd[4 + a])) return 0;
    }

    uint64_t N[4];
    for (int i = 0; i < 4; i++) N[i] = (uint64_t)kd[1 + i];
    /* iteration space and the part of it the collapsed loops expose */
    uint64_t I = N[0] * N[1] * N[2] * N[3];
    uint64_t TH = (uint64_t)T * (uint64_t)H;  /* hardware threads the launch asks for */
    uint64_t Pc = 1, R = 1, busy, waves, n_par;
    if (x == 0) {
        /* combined directive: loops 0..c-1 collapsed, the rest serial */
        for (int i = 0; i < c; i++) Pc *= N[i];
        for (int i = (int)c; i < 4; i++) R *= N[i];
        busy = TH < Pc ? TH : Pc;        /* threads that get work */
        waves = Pc / TH + (Pc % TH != 0);/* rounds of collapsed iterations per thread */
        n_par = (uint64_t)c;             /* loops collapsed into parallel work */
    } else {
        /* teams over loops 0..d-1, a team's threads over loops x..x+c-1 */
        uint64_t Pt = 1, Pf = 1;
        for (int i = 0; i < d; i++) Pt *= N[i];
        for (int i = (int)x; i < x + c; i++) Pf *= N[i];
        for (int i = (int)d; i < x; i++) R *= N[i];
        for (int i = (int)(x + c); i < 4; i++) R *= N[i];
        Pc = Pt * Pf;
        uint64_t bt = (uint64_t)T < Pt ? (uint64_t)T : Pt;
        uint64_t bf = (uint64_t)H < Pf ? (uint64_t)H : Pf;
        busy = bt * bf;
        waves = (Pt / (uint64_t)T + (Pt % (uint64_t)T != 0)) *
                (Pf / (uint64_t)H + (Pf % (uint64_t)H != 0));
        n_par = (uint64_t)(d + c);
    }
    uint64_t S = (uint64_t)E * I;             /* bytes of one array spanning the nest */
    uint64_t n_cls[4] = {0, 0, 0, 0};
    uint64_t ns = 0;
    for (int a = 0; a < A; a++) {
        n_cls[vd[4 + a]] += 1;
        ns += (uint64_t)kd[7 + a];
    }
    /* data moved by the chosen map clauses: to -> host-to-device,
     * from -> device-to-host, tofrom -> both, alloc -> none */
    uint64_t h2d = S * (n_cls[CLS_TO] + n_cls[CLS_TOFROM]);
    uint64_t d2h = S * (n_cls[CLS_FROM] + n_cls[CLS_TOFROM]);
    uint64_t line = 64u / (uint64_t)E;  /* elements per 64-byte line: cost of a strided walk */

    uint64_t u[NFEAT];
    u[0] = (uint64_t)D;
    u[1] = N[0]; u[2] = N[1]; u[3] = N[2]; u[4] = N[3];
    u[5] = I;
    u[6] = n_par;
    u[7] = Pc;
    u[8] = R;
    u[9] = (uint64_t)T;
    u[10] = (uint64_t)H;
    u[11] = TH;
    u[12] = busy;
    u[13] = waves;
    u[14] = waves * R;
    u[15] = waves * TH - Pc;
    u[16] = (uint64_t)A;
    u[17] = (uint64_t)E;
    u[18] = S;
    u[19] = n_cls[CLS_TO];
    u[20] = n_cls[CLS_FROM];
    u[21] = n_cls[CLS_TOFROM];
    u[22] = n_cls[CLS_ALLOC];
    u[23] = h2d;
    u[24] = d2h;
    u[25] = h2d + d2h;
    u[26] = ns;
    u[27] = S * (uint64_t)A;
    u[28] = S * ((uint64_t)A - ns) + line * S * ns;
    u[29] = (uint64_t)fpi * I;
    u[30] = (uint64_t)fpi;
    u[31] = S * n_cls[CLS_ALLOC];
    for (int j = 0; j < NFEAT; j++) f[j] = (int64_t)u[j];
    return 1;
}

/* Feature extraction over all variants. invalid may be NULL. */
void oracle_featurize(const int64_t *kdesc, const int64_t *vdesc, int64_t n_k, int64_t n_v,
                      int64_t *feat, uint8_t *invalid)
{
    for (int64_t i = 0; i < n_v; i++) {
        int ok = featurize_row(kdesc, vdesc + i * VD_COLS, n_k, feat + i * NFEAT);
        if (invalid) invalid[i] = (uint8_t)(!ok);
    }
}

/* The Z-score standardization of section 5.3 (the only transform the paper
 * applies to its data), taken on log2(1 + f): per-feature mean and
 * population standard deviation over a calibration sample. A feature that
 * takes a single value over the sample gets mean log2(1 + value) and
 * deviation 1, so it maps to exactly 0 (summing n copies of an inexact
 * logarithm would otherwise leave a deviation of rounding noise). A zero
 * deviation is likewise replaced by 1. */
void oracle_zscore_fit(const int64_t *feat, int64_t n, double *mu, double *sigma)
{
    for (int j = 0; j < NFEAT; j++) {
        int constant = 1;
        for (int64_t i = 1; i < n; i++) constant &= (feat[i * NFEAT + j] == feat[j]);
        if (n > 0 && constant) {
            mu[j] = log2((double)feat[j] + 1.0);
            sigma[j] = 1.0;
            continue;
        }
        double s = 0.0;
        for (int64_t i = 0; i < n; i++) s += log2((double)feat[i * NFEAT + j] + 1.0);
        double m = n > 0 ? s / (double)n : 0.0;
        double q = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double d = log2((double)feat[i * NFEAT + j] + 1.0) - m;
            q += d * d;
        }
        double sd = n > 0 ? sqrt(q / (double)n) : 0.0;
        mu[j] = m;
        sigma[j] = sd > 0.0 ? sd : 1.0;
    }
}

/* x_j = (log2(1 + f_j) - mu_j) / sigma_j */
static void normalize_row(const int64_t *f, const double *mu, const double *sigma, double *x)
{
    for (int j = 0; j < NFEAT; j++) x[j] = (log2((double)f[j] + 1.0) - mu[j]) / sigma[j];
}

void oracle_normalize(const int64_t *feat, int64_t n, const double *mu, const double *sigma,
                      double *x)
{
    for (int64_t i = 0; i < n; i++) normalize_row(feat + i * NFEAT, mu, sigma, x + i * NFEAT);
}

/* Offset of layer l's weight block in the concatenated parameter vector
 * [W_0 (out x in, row-major), b_0, W_1, b_1, ...]. */
static int64_t layer_offset(const int32_t *widths, int l)
{
    int64_t off = 0;
    for (int i = 0; i < l; i++) off += (int64_t)widths[i + 1] * widths[i] + widths[i + 1];
    return off;
}

/*
 * The fully-connected regression network of section 5.3 on one row:
 * h_0 = x; z_l = W_l h_{l-1} + b_l; h_l = act(z_l) on hidden layers; the last
 * layer is linear and its single output is the predicted log-runtime.
 * act = 0: ReLU, act = 1: identity (a linear network, used by the tests).
 * zs (optional) receives every layer's pre-activation, concatenated.
 */
static void forward_row(const int32_t *widths, int n_layers, const double *params, int act,
                        const double *x, double *buf_a, double *buf_b, double *zs, double *y)
{
    const double *h = x;
    double *out = buf_a;
    int64_t zoff = 0;
    for (int l = 0; l < n_layers; l++) {
        int fin = widths[l], fout = widths[l + 1];
        const double *W = params + layer_offset(widths, l);
        const double *b = W + (int64_t)fout * fin;
        for (int o = 0; o < fout; o++) {
            double z = b[o];
            for (int k = 0; k < fin; k++) z += W[(int64_t)o * fin + k] * h[k];
            if (zs) zs[zoff + o] = z;
            int hidden = l + 1 < n_layers;
            out[o] = (hidden && act == 0) ? (z > 0.0 ? z : 0.0) : z;
        }
        zoff += fout;
        h = out;
        out = (out == buf_a) ? buf_b : buf_a;
    }
    *y = h[0];
}

static int max_width(const int32_t *widths, int n_widths)
{
    int m = 0;
    for (int i = 0; i < n_widths; i++) m = widths[i] > m ? widths[i] : m;
    return m;
}

/* Network prediction for n rows of x [n, widths[0]]. */
int oracle_forward(const int32_t *widths, int n_widths, const double *params, int act,
                   const double *x, int64_t n, double *y)
{
    int nl = n_widths - 1, mw = max_width(widths, n_widths);
    if (nl < 1 || widths[nl] != 1) return -1;
    double *a = malloc(sizeof(double) * mw), *b = malloc(sizeof(double) * mw);
    if (!a || !b) { free(a); free(b); return -4; }
    for (int64_t i = 0; i < n; i++)
        forward_row(widths, nl, params, act, x + i * widths[0], a, b, NULL, y + i);
    free(a);
    free(b);
    return 0;
}

/*
 * Per-kernel selection of the prediction flow (section 3: predicted runtimes
 * are sorted and the best N variants kept; here N = 1). For every segment
 * [offsets[k], offsets[k+1]) the lowest predicted runtime wins, the lowest
 * variant index among equal predictions, NaN and invalid variants never win,
 * -0 equals +0, and an empty or all-excluded segment gives -1.
 */
void oracle_argmin(const double *pred, const uint8_t *invalid, const int64_t *offsets,
                   int64_t n_k, int64_t *best)
{
    for (int64_t k = 0; k < n_k; k++) {
        int64_t b = -1;
        for (int64_t i = offsets[k]; i < offsets[k + 1]; i++) {
            if (isnan(pred[i]) || (invalid && invalid[i])) continue;
            if (b == -1 || pred[i] < pred[b]) b = i;
        }
        best[k] = b;
    }
}

/* The top-N list of the prediction flow for each segment: (prediction,
 * index) ascending, excluded variants dropped, padded with -1. Selection by
 * repeated minimum keeps it a direct transcription of "lowest first, lowest
 * index on ties". out is [n_k, N]. */
void oracle_topn(const double *pred, const uint8_t *invalid, const int64_t *offsets,
                 int64_t n_k, int N, int64_t *out)
{
    for (int64_t k = 0; k < n_k; k++) {
        int64_t *row = out + k * N;
        for (int r = 0; r < N; r++) {
            int64_t b = -1;
            for (int64_t i = offsets[k]; i < offsets[k + 1]; i++) {
                if (isnan(pred[i]) || (invalid && invalid[i])) continue;
                int taken = 0;
                for (int q = 0; q < r; q++) taken |= (row[q] == i);
                if (taken) continue;
                if (b == -1 || pred[i] < pred[b]) b = i;
            }
            row[r] = b;
        }
    }
}

/* Mean squared error (1/B) sum (pred - y)^2: the square of the RMSE of
 * section 5.3, which has the same minimizer. */
double oracle_mse(const double *pred, const double *y, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double d = pred[i] - y[i];
        s += d * d;
    }
    return n > 0 ? s / (double)n : 0.0;
}

/*
 * Loss and gradient of the MSE with respect to every weight and bias, by the
 * chain rule through the network: delta_L = (2/B)(yhat - y);
 * dW_l = delta_l^T h_{l-1}; db_l = sum over the batch of delta_l;
 * delta_{l-1} = (delta_l W_l) * [z_{l-1} > 0] for ReLU (derivative 0 at 0),
 * or without the mask for the identity activation. grads has the parameter
 * layout. Returns 0, or -4 on allocation failure.
 */
int oracle_loss_grad(const int32_t *widths, int n_widths, const double *params, int act,
                     const double *x, const double *y, int64_t n, double *grads, double *loss)
{
    int nl = n_widths - 1, mw = max_width(widths, n_widths);
    if (nl < 1 || widths[nl] != 1) return -1;
    int64_t zlen = 0, np = layer_offset(widths, nl);
    for (int l = 1; l <= nl; l++) zlen += widths[l];
    double *zs = malloc(sizeof(double) * zlen);
    double *a = malloc(sizeof(double) * mw), *b = malloc(sizeof(double) * mw);
    double *hprev = malloc(sizeof(double) * mw);
    double *dcur = malloc(sizeof(double) * mw), *dnext = malloc(sizeof(double) * mw);
    if (!zs || !a || !b || !hprev || !dcur || !dnext) {
        free(zs); free(a); free(b); free(hprev); free(dcur); free(dnext);
        return -4;
    }
    memset(grads, 0, sizeof(double) * np);
    double sse = 0.0;
    for (int64_t i = 0; i < n; i++) {
        const double *xi = x + i * widths[0];
        double yhat;
        forward_row(widths, nl, params, act, xi, a, b, zs, &yhat);
        double r = yhat - y[i];
        sse += r * r;
        dcur[0] = 2.0 * r / (double)n;
        /* walk the layers from the output back to the input */
        int64_t zoff_end = zlen;
        for (int l = nl - 1; l >= 0; l--) {
            int fin = widths[l], fout = widths[l + 1];
            int64_t zoff = zoff_end - fout;           /* z_l lives at zs[zoff .. zoff+fout) */
            const double *W = params + layer_offset(widths, l);
            double *gW = grads + layer_offset(widths, l);
            double *gb = gW + (int64_t)fout * fin;
            /* input of layer l: x for l = 0, else act(z_{l-1}) */
            if (l == 0) {
                for (int k = 0; k < fin; k++) hprev[k] = xi[k];
            } else {
                const double *zp = zs + zoff - fin;
                for (int k = 0; k < fin; k++)
                    hprev[k] = act == 0 ? (zp[k] > 0.0 ? zp[k] : 0.0) : zp[k];
            }
            for (int o = 0; o < fout; o++) {
                gb[o] += dcur[o];
                for (int k = 0; k < fin; k++) gW[(int64_t)o * fin + k] += dcur[o] * hprev[k];
            }
            if (l > 0) {
                const double *zp = zs + zoff - fin;
                for (int k = 0; k < fin; k++) {
                    double s = 0.0;
                    for (int o = 0; o < fout; o++) s += dcur[o] * W[(int64_t)o * fin + k];
                    dnext[k] = (act == 0 && !(zp[k] > 0.0)) ? 0.0 : s;
                }
                for (int k = 0; k < fin; k++) dcur[k] = dnext[k];
            }
            zoff_end = zoff;
        }
    }
    if (loss) *loss = n > 0 ? sse / (double)n : 0.0;
    free(zs); free(a); free(b); free(hprev); free(dcur); free(dnext);
    return 0;
}

/* Euclidean norm of a gradient vector. */
double oracle_l2norm(const double *g, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += g[i] * g[i];
    return sqrt(s);
}

/* One Adam step (Kingma and Ba, the optimizer the paper evaluates in
 * section 5.3): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 * w <- w - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps); t counts from 1. */
void oracle_adam(double *w, double *m, double *v, const double *g, int64_t n, int64_t t,
                 double lr, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/*
 * Data analysis of section 4.1.2: the map class of each variable a kernel
 * uses, from what happens to it before, during and after the kernel. The
 * access bits: 1 assigned before the kernel, 2 read within it, 4 written
 * (assigned or updated) within it, 8 accessed after it, 16 declared within
 * it. Classes (codes shared with the descriptors' data classes):
 *   0 alloc   - first assigned within the kernel, not needed after it;
 *   1 to      - assigned before and only read within (not modified);
 *   2 from    - updated within and accessed after, not assigned before;
 *   3 tofrom  - assigned before, updated within and accessed after;
 *   4 private - declared within the kernel;
 *   5 none    - neither read nor written within (not a kernel variable).
 * Patterns the five definitions leave open take the choice that moves the
 * data the kernel may need: a variable read within but never modified is
 * "to" even without an assignment before; one assigned before, updated and
 * read within but not needed after is "to"; one assigned before and only
 * written within (its old value never read) and not needed after is alloc.
 */
int oracle_map_class(int bits)
{
    int before = bits & 1, rd = (bits >> 1) & 1, wr = (bits >> 2) & 1, after = (bits >> 3) & 1;
    if (bits & 16) return 4;
    if (!rd && !wr) return 5;
    if (!wr) return 1;
    if (after) return before ? 3 : 2;
    return (before && rd) ? 1 : 0;
}

/*
 * Per kernel k (variables [var_off[k], var_off[k+1])): the class of every
 * variable, and the bytes of the enter-data directive's transfers (to and
 * tofrom variables), of the exit-data directive's (from and tofrom), and of
 * mapping every variable the kernel uses (classes 0-3) to and from the GPU,
 * the untransformed code of section 5.1's first experiment.
 */
void oracle_classify(const uint8_t *access, const int64_t *bytes, const int64_t *var_off,
                     int64_t n_k, uint8_t *cls, int64_t *enter, int64_t *exit_, int64_t *naive)
{
    for (int64_t k = 0; k < n_k; k++) {
        int64_t e = 0, x = 0, nv = 0;
        for (int64_t i = var_off[k]; i < var_off[k + 1]; i++) {
            int c = oracle_map_class(access[i]);
            cls[i] = (uint8_t)c;
            if (c == 1 || c == 3) e += bytes[i];
            if (c == 2 || c == 3) x += bytes[i];
            if (c <= 3) nv += 2 * bytes[i];
        }
        enter[k] = e;
        exit_[k] = x;
        naive[k] = nv;
    }
}

/*
 * Variant generation of section 4.1.3 for one kernel with n collapsible
 * loops (1 <= n <= 4; any other n gives no variant). Loop 0 is always
 * distributed over the teams. The parallel-for directive sits at loop x:
 * at x = 0 it merges with teams distribute into one combined directive
 * whose collapse c runs over 1..n (no separate teams collapse, d = 0); at
 * 1 <= x < n teams distribute collapses d in 1..x loops and parallel for
 * collapses c in 1..n-x. Every placement takes each schedule whose bit is
 * set in sched_mask (bit 0 static, 1 dynamic, 2 guided) and each of the two
 * data-transfer options. Rows [x, d, c, schedule, data] in that nesting
 * order are written to out (if not NULL); the count is returned.
 */
int64_t oracle_enumerate(int n, int sched_mask, int64_t *out)
{
    int64_t count = 0;
    if (n < 1 || n > 4) return 0;
    for (int x = 0; x < n; x++) {
        int d_lo = x == 0 ? 0 : 1, d_hi = x == 0 ? 0 : x;
        int c_hi = x == 0 ? n : n - x;
        for (int d = d_lo; d <= d_hi; d++)
            for (int c = 1; c <= c_hi; c++)
                for (int sch = 0; sch < 3; sch++) {
                    if (!((sched_mask >> sch) & 1)) continue;
                    for (int data = 0; data < 2; data++) {
                        if (out) {
                            int64_t *r = out + count * 5;
                            r[0] = x; r[1] = d; r[2] = c; r[3] = sch; r[4] = data;
                        }
                        count++;
                    }
                }
    }
    return count;
}

/*
 * A generated variant (section 4.1.3) as a cost-model descriptor row. gen row
 * [k, x, d, c, schedule, data] -> vdesc row [k, c + 8 x + 64 d + 512 schedule,
 * teams, threads, m0..m3]. The generated directives carry no num_teams or
 * thread_limit clause, so teams and threads are the launch the target's
 * runtime makes by default (given by the caller). The two data-transfer
 * options: 0 maps every array with the class the data analysis gives it
 * (section 4.1.2: enter/exit data of exactly what the kernel needs), 1 maps
 * every array tofrom (the untransformed code that moves everything both
 * ways). Arrays past the kernel's A are left 0.
 */
void oracle_lower_variants(const int64_t *kdesc, const int64_t *gen, int64_t n_v, int64_t teams,
                           int64_t threads, int64_t *vdesc)
{
    for (int64_t i = 0; i < n_v; i++) {
        const int64_t *g = gen + i * 6;
        int64_t *v = vdesc + i * VD_COLS;
        const int64_t *kd = kdesc + g[0] * KD_COLS;
        v[0] = g[0];
        v[1] = g[3] + 8 * g[1] + 64 * g[2] + 512 * g[4];
        v[2] = teams;
        v[3] = threads;
        for (int a = 0; a < 4; a++) v[4 + a] = a < kd[5] ? (g[5] == 0 ? kd[12 + a] : CLS_TOFROM) : 0;
    }
}

/*
 * RMSprop (the optimizer section 5.3 selects; Hinton's lecture notes), with
 * the weight decay of section 5.3 entering as an L2 term of the gradient:
 * g' = g + wd w; v <- alpha v + (1 - alpha) g'^2; w <- w - lr g' / (sqrt(v) + eps).
 */
void oracle_rmsprop(double *w, double *v, const double *g, int64_t n, double lr, double alpha,
                    double eps, double wd)
{
    for (int64_t i = 0; i < n; i++) {
        double gi = g[i] + wd * w[i];
        v[i] = alpha * v[i] + (1.0 - alpha) * gi * gi;
        w[i] -= lr * gi / (sqrt(v[i]) + eps);
    }
}

/*
 * The whole prediction flow for many kernels: featurize every variant,
 * standardize, predict, and pick each kernel's best variant. Kernels are
 * independent, so they are spread over threads (n_threads <= 0: the OpenMP
 * default). A variant takes part only if it is valid and its kernel id names
 * the segment it sits in. pred (optional) receives every variant's
 * prediction, NaN for the variants that take no part.
 */
int oracle_rank(const int64_t *kdesc, const int64_t *vdesc, const int64_t *offsets,
                int64_t n_k, int64_t n_v, const int32_t *widths, int n_widths,
                const double *params, const double *mu, const double *sigma,
                int64_t *best, double *pred, int n_threads)
{
    int nl = n_widths - 1, mw = max_width(widths, n_widths);
    if (nl < 1 || widths[0] != NFEAT || widths[nl] != 1) return -1;
    if (offsets[0] != 0 || offsets[n_k] != n_v) return -2;
    int status = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        double *a = malloc(sizeof(double) * mw), *b = malloc(sizeof(double) * mw);
        double x[NFEAT];
        int64_t f[NFEAT];
        if (!a || !b) {
#pragma omp atomic write
            status = -4;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t k = 0; k < n_k; k++) {
            if (!a || !b) continue;
            int64_t bi = -1;
            double bv = 0.0;
            for (int64_t i = offsets[k]; i < offsets[k + 1]; i++) {
                int ok = vdesc[i * VD_COLS] == k &&
                         featurize_row(kdesc, vdesc + i * VD_COLS, n_k, f);
                double yi = NAN;
                if (ok) {
                    normalize_row(f, mu, sigma, x);
                    forward_row(widths, nl, params, 0, x, a, b, NULL, &yi);
                }
                if (pred) pred[i] = yi;
                if (!ok || isnan(yi)) continue;
                if (bi == -1 || yi < bv) { bi = i; bv = yi; }
            }
            best[k] = bi;
        }
        free(a);
        free(b);
    }
    return status;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
