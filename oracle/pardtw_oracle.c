/*
 * pardtw_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of exact DTW as
 * used by Parallelized Diagonal DTW (ParDTW). Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library; the GPU
 * product path never calls it, links it, or shares code with it.
 *
 * What it computes (Yang, Shaw & Tsai, "A Study of Parallelizable Alternatives
 * to Dynamic Time Warping for Aligning Long Sequences"):
 *
 *  - Pairwise cost: cosine distance between feature frames (Sec. IV,
 *    experimental setup): C[i,j] = 1 - <x_i, y_j> / (|x_i| |y_j|).
 *    A zero frame is taken to normalise to the zero vector, so its cost is 1.
 *  - Accumulated cost: standard DTW with (query, reference) steps
 *    {(1,1), (1,2), (2,1)} and multiplicative weights {2, 3, 3} (Sec. V,
 *    baseline DTW); ParDTW computes exactly this result (Sec. II-D, Sec. V).
 *    The weight multiplies the cost of the cell a step lands on. The start
 *    cell carries weight 1: D[0,0] = C[0,0]. For every other cell
 *        D[i,j] = min( D[i-1,j-1] + 2 C[i,j],
 *                      D[i-1,j-2] + 3 C[i,j],
 *                      D[i-2,j-1] + 3 C[i,j] )
 *    with out-of-range predecessors equal to +inf. The backtrace code of a
 *    cell is the index of the winning candidate, where an exact tie goes to
 *    the lowest index (strict-less updates in the printed step order); a cell
 *    whose three candidates are all +inf gets code 3, and so does (0,0).
 *    Rows are swept top to bottom; a row needs only the two rows above it.
 *  - Backtrace: follow the stored codes from (N-1, M-1) back to (0,0)
 *    (Sec. II-D keeps the backtrace matrix and backtraces at the end).
 *  - Gradient of the DTW cost with the optimal path held fixed, for the
 *    differentiable form (the paper motivates backpropagation through the
 *    optimal path in Sec. I).
 *
 * All arithmetic is IEEE double; inputs are the FP32 feature bits.
 * Build: gcc -O2 -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CODE_DIAG 0  /* step (1,1), weight 2 */
#define CODE_RIGHT 1 /* step (1,2), weight 3 */
#define CODE_DOWN 2  /* step (2,1), weight 3 */
#define CODE_NONE 3  /* origin or unreachable */

static const int STEP_DI[3] = {1, 1, 2};
static const int STEP_DJ[3] = {1, 2, 1};
static const double STEP_W[3] = {2.0, 3.0, 3.0};

/* Unit-normalise every row of a (rows x d) FP32 matrix into FP64. */
static double* unit_rows(const float* a, int64_t rows, int64_t d) {
    double* out = (double*)malloc(sizeof(double) * (size_t)(rows * d));
    if (!out) return NULL;
    for (int64_t r = 0; r < rows; ++r) {
        double s = 0.0;
        for (int64_t k = 0; k < d; ++k) {
            double v = (double)a[r * d + k];
            s += v * v;
        }
        double nrm = sqrt(s);
        for (int64_t k = 0; k < d; ++k)
            out[r * d + k] = nrm > 0.0 ? (double)a[r * d + k] / nrm : 0.0;
    }
    return out;
}

/* One row of cosine distances: crow[j] = 1 - <xh_i, yh_j>. */
static void cost_row(const double* xh_i, const double* yh, int64_t m, int64_t d, double* crow) {
    for (int64_t j = 0; j < m; ++j) {
        double dot = 0.0;
        for (int64_t k = 0; k < d; ++k) dot += xh_i[k] * yh[j * d + k];
        crow[j] = 1.0 - dot;
    }
}

/* Full (n x m) cosine-distance matrix in FP64. Returns 0 on success. */
int oracle_cost(const float* X, const float* Y, int64_t n, int64_t m, int64_t d, double* C) {
    double* xh = unit_rows(X, n, d);
    double* yh = unit_rows(Y, m, d);
    if (!xh || !yh) { free(xh); free(yh); return -1; }
    for (int64_t i = 0; i < n; ++i) cost_row(xh + i * d, yh, m, d, C + i * m);
    free(xh);
    free(yh);
    return 0;
}

/* The DP for one row i given the two rows above (prev1 = row i-1, prev2 =
 * row i-2; NULL when that row does not exist) and the cost row. Writes the
 * accumulated costs into cur and the codes into bp_row. When cand is not NULL
 * it receives the three candidate totals per cell (3*m doubles). */
static void dp_row_range(int64_t i, int64_t j0, int64_t j1, const double* crow, const double* prev1,
                         const double* prev2, double* cur, int8_t* bp_row, double* cand) {
    for (int64_t j = j0; j < j1; ++j) {
        double c = crow[j];
        double cd[3];
        cd[0] = (prev1 && j >= 1) ? prev1[j - 1] + STEP_W[0] * c : INFINITY;
        cd[1] = (prev1 && j >= 2) ? prev1[j - 2] + STEP_W[1] * c : INFINITY;
        cd[2] = (prev2 && j >= 1) ? prev2[j - 1] + STEP_W[2] * c : INFINITY;
        double best = cd[0];
        int code = CODE_DIAG;
        if (cd[1] < best) { best = cd[1]; code = CODE_RIGHT; }
        if (cd[2] < best) { best = cd[2]; code = CODE_DOWN; }
        if (isinf(best) && best > 0) code = CODE_NONE;
        if (i == 0 && j == 0) { best = c; code = CODE_NONE; }
        cur[j] = best;
        if (bp_row) bp_row[j] = (int8_t)code;
        if (cand) { cand[3 * j] = cd[0]; cand[3 * j + 1] = cd[1]; cand[3 * j + 2] = cd[2]; }
    }
}

static void dp_row(int64_t i, int64_t m, const double* crow, const double* prev1, const double* prev2,
                   double* cur, int8_t* bp_row, double* cand) {
    dp_row_range(i, 0, m, crow, prev1, prev2, cur, bp_row, cand);
}

/* DP over a given FP64 cost matrix. D_opt (n*m) is optional; BP (n*m int8)
 * is required. *total receives D[n-1, m-1] (+inf when no path exists). */
int oracle_dtw_matrix(const double* C, int64_t n, int64_t m, double* D_opt, int8_t* BP, double* total) {
    if (n <= 0 || m <= 0) return -1;
    double* rows = (double*)malloc(sizeof(double) * (size_t)(3 * m));
    if (!rows) return -1;
    double* r[3] = {rows, rows + m, rows + 2 * m};
    for (int64_t i = 0; i < n; ++i) {
        double* cur = r[i % 3];
        const double* p1 = i >= 1 ? r[(i - 1) % 3] : NULL;
        const double* p2 = i >= 2 ? r[(i - 2) % 3] : NULL;
        dp_row(i, m, C + i * m, p1, p2, cur, BP + i * m, NULL);
        if (D_opt) memcpy(D_opt + i * m, cur, sizeof(double) * (size_t)m);
    }
    *total = r[(n - 1) % 3][m - 1];
    free(rows);
    return 0;
}

/* Same DP, FP64 arithmetic, over an FP32 cost matrix (every FP32 value is
 * exact in FP64). Used to test the GPU dynamic program on its own. */
int oracle_dtw_matrix_f32(const float* C, int64_t n, int64_t m, double* D_opt, int8_t* BP, double* total) {
    if (n <= 0 || m <= 0) return -1;
    double* rows = (double*)malloc(sizeof(double) * (size_t)(4 * m));
    if (!rows) return -1;
    double* r[3] = {rows, rows + m, rows + 2 * m};
    double* crow = rows + 3 * m;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) crow[j] = (double)C[i * m + j];
        double* cur = r[i % 3];
        const double* p1 = i >= 1 ? r[(i - 1) % 3] : NULL;
        const double* p2 = i >= 2 ? r[(i - 2) % 3] : NULL;
        dp_row(i, m, crow, p1, p2, cur, BP + i * m, NULL);
        if (D_opt) memcpy(D_opt + i * m, cur, sizeof(double) * (size_t)m);
    }
    *total = r[(n - 1) % 3][m - 1];
    free(rows);
    return 0;
}

/* DP from features with the cost computed row by row (no n*m cost matrix is
 * held, so this runs at the long-sequence sizes). BP (n*m int8) required. */
int oracle_dtw_features(const float* X, const float* Y, int64_t n, int64_t m, int64_t d, int8_t* BP,
                        double* total) {
    if (n <= 0 || m <= 0 || d <= 0) return -1;
    double* xh = unit_rows(X, n, d);
    double* yh = unit_rows(Y, m, d);
    double* rows = (double*)malloc(sizeof(double) * (size_t)(4 * m));
    if (!xh || !yh || !rows) { free(xh); free(yh); free(rows); return -1; }
    double* r[3] = {rows, rows + m, rows + 2 * m};
    double* crow = rows + 3 * m;
    for (int64_t i = 0; i < n; ++i) {
        cost_row(xh + i * d, yh, m, d, crow);
        double* cur = r[i % 3];
        const double* p1 = i >= 1 ? r[(i - 1) % 3] : NULL;
        const double* p2 = i >= 2 ? r[(i - 2) % 3] : NULL;
        dp_row(i, m, crow, p1, p2, cur, BP + i * m, NULL);
    }
    *total = r[(n - 1) % 3][m - 1];
    free(xh); free(yh); free(rows);
    return 0;
}

/* oracle_dtw_features with the columns of each row split over `threads`
 * OpenMP threads. A cell needs only the two rows above it, so the cells of a
 * row are independent; every cell runs the same arithmetic as in the serial
 * sweep, and BP and total are bit-identical to it. Used to time the oracle on
 * all host cores. */
int oracle_dtw_features_mt(const float* X, const float* Y, int64_t n, int64_t m, int64_t d, int8_t* BP,
                           double* total, int threads) {
    if (n <= 0 || m <= 0 || d <= 0 || threads <= 0) return -1;
    double* xh = unit_rows(X, n, d);
    double* yh = unit_rows(Y, m, d);
    double* rows = (double*)malloc(sizeof(double) * (size_t)(4 * m));
    if (!xh || !yh || !rows) { free(xh); free(yh); free(rows); return -1; }
    double* r[3] = {rows, rows + m, rows + 2 * m};
    double* crow = rows + 3 * m;
    const int64_t blocks = 4 * (int64_t)threads < m ? 4 * (int64_t)threads : m;
#pragma omp parallel num_threads(threads)
    for (int64_t i = 0; i < n; ++i) {
        double* cur = r[i % 3];
        const double* p1 = i >= 1 ? r[(i - 1) % 3] : NULL;
        const double* p2 = i >= 2 ? r[(i - 2) % 3] : NULL;
        /* the loop's implicit barrier ends row i before row i+1 starts */
#pragma omp for schedule(static)
        for (int64_t b = 0; b < blocks; ++b) {
            const int64_t j0 = b * m / blocks, j1 = (b + 1) * m / blocks;
            cost_row(xh + i * d, yh + j0 * d, j1 - j0, d, crow + j0);
            dp_row_range(i, j0, j1, crow, p1, p2, cur, BP + i * m, NULL);
        }
    }
    *total = r[(n - 1) % 3][m - 1];
    free(xh); free(yh); free(rows);
    return 0;
}

/* Re-sweep from features and record, for each requested cell (ci[k], cj[k]),
 * the three FP64 candidate totals (cand[3k..3k+2]) and the cell's FP64
 * accumulated cost (dval[k]). Requested cells must be sorted by row. When
 * C32 is not NULL the sweep uses that FP32 cost matrix instead of features. */
int oracle_probe(const float* X, const float* Y, const float* C32, int64_t n, int64_t m, int64_t d,
                 const int64_t* ci, const int64_t* cj, int64_t k, double* cand, double* dval) {
    if (n <= 0 || m <= 0) return -1;
    double* xh = NULL;
    double* yh = NULL;
    if (!C32) {
        xh = unit_rows(X, n, d);
        yh = unit_rows(Y, m, d);
        if (!xh || !yh) { free(xh); free(yh); return -1; }
    }
    double* rows = (double*)malloc(sizeof(double) * (size_t)(4 * m));
    double* rc = (double*)malloc(sizeof(double) * (size_t)(3 * m));
    if (!rows || !rc) { free(xh); free(yh); free(rows); free(rc); return -1; }
    double* r[3] = {rows, rows + m, rows + 2 * m};
    double* crow = rows + 3 * m;
    int64_t q = 0;
    for (int64_t i = 0; i < n && q < k; ++i) {
        if (C32) for (int64_t j = 0; j < m; ++j) crow[j] = (double)C32[i * m + j];
        else cost_row(xh + i * d, yh, m, d, crow);
        double* cur = r[i % 3];
        const double* p1 = i >= 1 ? r[(i - 1) % 3] : NULL;
        const double* p2 = i >= 2 ? r[(i - 2) % 3] : NULL;
        dp_row(i, m, crow, p1, p2, cur, NULL, rc);
        while (q < k && ci[q] == i) {
            int64_t j = cj[q];
            cand[3 * q] = rc[3 * j];
            cand[3 * q + 1] = rc[3 * j + 1];
            cand[3 * q + 2] = rc[3 * j + 2];
            dval[q] = cur[j];
            ++q;
        }
        if (q < k && ci[q] < i) { free(xh); free(yh); free(rows); free(rc); return -2; }
    }
    free(xh); free(yh); free(rows); free(rc);
    return q == k ? 0 : -3;
}

/* Backtrace from (n-1, m-1). Writes the path forward (from (0,0)) as int32
 * (i, j) pairs into path (capacity min(n, m) pairs) and returns its length,
 * or 0 when the end cell is unreachable. */
int64_t oracle_backtrace(const int8_t* BP, int64_t n, int64_t m, int32_t* path) {
    int64_t cap = n < m ? n : m;
    int64_t i = n - 1, j = m - 1, len = 0;
    int32_t* rev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * cap));
    if (!rev) return -1;
    for (;;) {
        if (len >= cap) { free(rev); return -1; }
        rev[2 * len] = (int32_t)i;
        rev[2 * len + 1] = (int32_t)j;
        ++len;
        if (i == 0 && j == 0) break;
        int code = BP[i * m + j];
        if (code < 0 || code > 2) { free(rev); return 0; }
        i -= STEP_DI[code];
        j -= STEP_DJ[code];
        if (i < 0 || j < 0) { free(rev); return -1; }
    }
    for (int64_t l = 0; l < len; ++l) {
        path[2 * l] = rev[2 * (len - 1 - l)];
        path[2 * l + 1] = rev[2 * (len - 1 - l) + 1];
    }
    free(rev);
    return len;
}

/* FP64 cost of a given path: C[p_0] + sum_l w(p_l - p_{l-1}) C[p_l], with the
 * cost computed from features exactly as in cost_row. Returns NAN for an
 * illegal path. */
double oracle_path_cost(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                        const int32_t* path, int64_t len) {
    if (len <= 0) return NAN;
    double total = 0.0;
    for (int64_t l = 0; l < len; ++l) {
        int64_t i = path[2 * l], j = path[2 * l + 1];
        if (i < 0 || i >= n || j < 0 || j >= m) return NAN;
        double w = 1.0;
        if (l > 0) {
            int64_t di = i - path[2 * (l - 1)], dj = j - path[2 * (l - 1) + 1];
            if (di == 1 && dj == 1) w = STEP_W[0];
            else if (di == 1 && dj == 2) w = STEP_W[1];
            else if (di == 2 && dj == 1) w = STEP_W[2];
            else return NAN;
        } else if (i != 0 || j != 0) {
            return NAN;
        }
        double* xh = unit_rows(X + i * d, 1, d);
        double* yh = unit_rows(Y + j * d, 1, d);
        if (!xh || !yh) { free(xh); free(yh); return NAN; }
        double c;
        cost_row(xh, yh, 1, d, &c);
        free(xh); free(yh);
        total += w * c;
    }
    if (path[2 * (len - 1)] != n - 1 || path[2 * (len - 1) + 1] != m - 1) return NAN;
    return total;
}

/* Gradient of J(P) = sum_l w_l c(x_{i_l}, y_{j_l}) with the path P held fixed,
 * scaled by g. With u = x/|x|, v = y/|y| and c = 1 - <u,v>:
 *   dc/dx = -(v - <u,v> u) / |x|,   dc/dy = -(u - <u,v> v) / |y|.
 * dX (n*d) and dY (m*d) are overwritten; rows and columns the path skips get
 * zero. A zero frame has zero gradient. */
int oracle_path_grad(const float* X, const float* Y, int64_t n, int64_t m, int64_t d,
                     const int32_t* path, int64_t len, double g, double* dX, double* dY) {
    memset(dX, 0, sizeof(double) * (size_t)(n * d));
    memset(dY, 0, sizeof(double) * (size_t)(m * d));
    for (int64_t l = 0; l < len; ++l) {
        int64_t i = path[2 * l], j = path[2 * l + 1];
        double w = 1.0;
        if (l > 0) {
            int64_t di = i - path[2 * (l - 1)], dj = j - path[2 * (l - 1) + 1];
            w = (di == 1 && dj == 1) ? 2.0 : 3.0;
        }
        double sx = 0.0, sy = 0.0;
        for (int64_t k = 0; k < d; ++k) {
            double a = (double)X[i * d + k], b = (double)Y[j * d + k];
            sx += a * a; sy += b * b;
        }
        double nx = sqrt(sx), ny = sqrt(sy);
        if (nx == 0.0 || ny == 0.0) continue;
        double uv = 0.0;
        for (int64_t k = 0; k < d; ++k) uv += ((double)X[i * d + k] / nx) * ((double)Y[j * d + k] / ny);
        for (int64_t k = 0; k < d; ++k) {
            double u = (double)X[i * d + k] / nx, v = (double)Y[j * d + k] / ny;
            dX[i * d + k] += g * w * (-(v - uv * u) / nx);
            dY[j * d + k] += g * w * (-(u - uv * v) / ny);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Subsequence DTW and the segment-level programs of Segmental DTW
 * (Sec. II-B to II-D: NSDTW and WSDTW).
 *
 * Subsequence DTW aligns a short query (a fragment of sequence A, rows i) with
 * the best-matching stretch of a long reference (sequence B, columns j). The
 * steps are the same (query, reference) steps (1,1), (1,2), (2,1), now with
 * multiplicative weights 1, 1, 2 (Sec. II-B), still applied to the cell a step
 * lands on. A path may begin anywhere on the first query row at no extra
 * charge: D[0,j] = C[0,j] (start cell weight 1, code 3). For i >= 1
 *     D[i,j] = min( D[i-1,j-1] + C[i,j],
 *                   D[i-1,j-2] + C[i,j],
 *                   D[i-2,j-1] + 2 C[i,j] )
 * with out-of-range predecessors +inf, exact ties to the lowest step index,
 * and code 3 where all three are +inf. The weights equal each step's advance
 * along the query, so every path from row 0 to row n-1 carries total weight n
 * and the scores S[j] = D[n-1,j] of different end columns are comparable.
 * ------------------------------------------------------------------------ */

static const double SUB_W[3] = {1.0, 1.0, 2.0};

static void sub_row(int64_t i, int64_t m, const double* crow, const double* prev1, const double* prev2,
                    double* cur, int8_t* bp_row, double* cand) {
    for (int64_t j = 0; j < m; ++j) {
        double c = crow[j];
        double cd[3];
        cd[0] = (prev1 && j >= 1) ? prev1[j - 1] + SUB_W[0] * c : INFINITY;
        cd[1] = (prev1 && j >= 2) ? prev1[j - 2] + SUB_W[1] * c : INFINITY;
        cd[2] = (prev2 && j >= 1) ? prev2[j - 1] + SUB_W[2] * c : INFINITY;
        double best = cd[0];
        int code = CODE_DIAG;
        if (cd[1] < best) { best = cd[1]; code = CODE_RIGHT; }
        if (cd[2] < best) { best = cd[2]; code = CODE_DOWN; }
        if (isinf(best) && best > 0) code = CODE_NONE;
        if (i == 0) { best = c; code = CODE_NONE; }  /* free start on the first query row */
        cur[j] = best;
        if (bp_row) bp_row[j] = (int8_t)code;
        if (cand) { cand[3 * j] = cd[0]; cand[3 * j + 1] = cd[1]; cand[3 * j + 2] = cd[2]; }
    }
}

/* Cost rows come from an FP64 matrix (C64), an FP32 matrix (C32, widened
 * exactly) or features (X, Y). D_opt (n*m) and BP (n*m) are optional; S (m)
 * receives the last row. */
static int sub_sweep(const double* C64, const float* C32, const float* X, const float* Y, int64_t n, int64_t m,
                     int64_t d, double* D_opt, int8_t* BP, double* S) {
    if (n <= 0 || m <= 0) return -1;
    double* xh = NULL;
    double* yh = NULL;
    if (!C64 && !C32) {
        xh = unit_rows(X, n, d);
        yh = unit_rows(Y, m, d);
        if (!xh || !yh) { free(xh); free(yh); return -1; }
    }
    double* rows = (double*)malloc(sizeof(double) * (size_t)(4 * m));
    if (!rows) { free(xh); free(yh); return -1; }
    double* r[3] = {rows, rows + m, rows + 2 * m};
    double* crow = rows + 3 * m;
    for (int64_t i = 0; i < n; ++i) {
        if (C64) memcpy(crow, C64 + i * m, sizeof(double) * (size_t)m);
        else if (C32) for (int64_t j = 0; j < m; ++j) crow[j] = (double)C32[i * m + j];
        else cost_row(xh + i * d, yh, m, d, crow);
        double* cur = r[i % 3];
        const double* p1 = i >= 1 ? r[(i - 1) % 3] : NULL;
        const double* p2 = i >= 2 ? r[(i - 2) % 3] : NULL;
        sub_row(i, m, crow, p1, p2, cur, BP ? BP + i * m : NULL, NULL);
        if (D_opt) memcpy(D_opt + i * m, cur, sizeof(double) * (size_t)m);
    }
    memcpy(S, r[(n - 1) % 3], sizeof(double) * (size_t)m);
    free(xh); free(yh); free(rows);
    return 0;
}

int oracle_subseq_matrix(const double* C, int64_t n, int64_t m, double* D_opt, int8_t* BP, double* S) {
    return sub_sweep(C, NULL, NULL, NULL, n, m, 0, D_opt, BP, S);
}

int oracle_subseq_matrix_f32(const float* C, int64_t n, int64_t m, double* D_opt, int8_t* BP, double* S) {
    return sub_sweep(NULL, C, NULL, NULL, n, m, 0, D_opt, BP, S);
}

int oracle_subseq_features(const float* X, const float* Y, int64_t n, int64_t m, int64_t d, int8_t* BP, double* S) {
    if (d <= 0) return -1;
    return sub_sweep(NULL, NULL, X, Y, n, m, d, NULL, BP, S);
}

/* Candidate totals and D at requested cells (sorted by row), as oracle_probe
 * does for DTW, from an FP32 cost matrix or from features. */
int oracle_subseq_probe(const float* X, const float* Y, const float* C32, int64_t n, int64_t m, int64_t d,
                        const int64_t* ci, const int64_t* cj, int64_t k, double* cand, double* dval) {
    if (n <= 0 || m <= 0) return -1;
    double* xh = NULL;
    double* yh = NULL;
    if (!C32) {
        xh = unit_rows(X, n, d);
        yh = unit_rows(Y, m, d);
        if (!xh || !yh) { free(xh); free(yh); return -1; }
    }
    double* rows = (double*)malloc(sizeof(double) * (size_t)(4 * m));
    double* rc = (double*)malloc(sizeof(double) * (size_t)(3 * m));
    if (!rows || !rc) { free(xh); free(yh); free(rows); free(rc); return -1; }
    double* r[3] = {rows, rows + m, rows + 2 * m};
    double* crow = rows + 3 * m;
    int64_t q = 0;
    for (int64_t i = 0; i < n && q < k; ++i) {
        if (C32) for (int64_t j = 0; j < m; ++j) crow[j] = (double)C32[i * m + j];
        else cost_row(xh + i * d, yh, m, d, crow);
        double* cur = r[i % 3];
        const double* p1 = i >= 1 ? r[(i - 1) % 3] : NULL;
        const double* p2 = i >= 2 ? r[(i - 2) % 3] : NULL;
        sub_row(i, m, crow, p1, p2, cur, NULL, rc);
        while (q < k && ci[q] == i) {
            int64_t j = cj[q];
            cand[3 * q] = rc[3 * j];
            cand[3 * q + 1] = rc[3 * j + 1];
            cand[3 * q + 2] = rc[3 * j + 2];
            dval[q] = cur[j];
            ++q;
        }
        if (q < k && ci[q] < i) { free(xh); free(yh); free(rows); free(rc); return -2; }
    }
    free(xh); free(yh); free(rows); free(rc);
    return q == k ? 0 : -3;
}

/* Backtrace of a subsequence path ending at (n-1, end): follow the codes up
 * to the first query row. Writes the path forward (capacity n pairs) and
 * returns its length, 0 when (n-1, end) is unreachable, -1 on malformed codes. */
int64_t oracle_subseq_backtrace(const int8_t* BP, int64_t n, int64_t m, int64_t end, int32_t* path) {
    if (end < 0 || end >= m) return 0;
    int64_t i = n - 1, j = end, len = 0;
    int32_t* rev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * n));
    if (!rev) return -1;
    for (;;) {
        if (len >= n) { free(rev); return -1; }
        rev[2 * len] = (int32_t)i;
        rev[2 * len + 1] = (int32_t)j;
        ++len;
        if (i == 0) break;
        int code = BP[i * m + j];
        if (code == CODE_NONE && len == 1) { free(rev); return 0; }
        if (code < 0 || code > 2) { free(rev); return -1; }
        i -= STEP_DI[code];
        j -= STEP_DJ[code];
        if (i < 0 || j < 0) { free(rev); return -1; }
    }
    for (int64_t l = 0; l < len; ++l) {
        path[2 * l] = rev[2 * (len - 1 - l)];
        path[2 * l + 1] = rev[2 * (len - 1 - l) + 1];
    }
    free(rev);
    return len;
}

/* Segment level (Sec. II-C steps 3-4; Sec. II-B for NSDTW). S is the
 * (nf x m) matrix whose row f holds fragment f's subsequence scores, one per
 * end column (the segment-level cost matrix).
 *
 * variant 0, NSDTW: each fragment independently ends at its lowest score
 *   (the first such column); total = sum of those scores.
 * variant 1, WSDTW: a path through S with (fragment, column) transitions
 *   (0,1), a free skip, and (1,hop), a match that pays S[f,j]:
 *       Dseg[f,j] = min( Dseg[f,j-1], Dseg[f-1,j-hop] + S[f,j] ),
 *   Dseg[f,-1] = +inf, Dseg[-1,j] = 0 for every j (the first fragment may end
 *   anywhere), Dseg[f-1,j-hop] = +inf for f >= 1 and j < hop. A match replaces
 *   the skip only when strictly smaller (the skip is the first term). The
 *   total is Dseg[nf-1,m-1]; backtracking from there, a match at (f,j) ends
 *   fragment f at column j and moves to (f-1, j-hop), a skip moves to (f, j-1).
 * ends[f] = -1 and total = +inf when no placement has a finite score.
 * Returns 0 on success. */
int oracle_segment_ends(const double* S, int64_t nf, int64_t m, int64_t hop, int variant, int64_t* ends,
                        double* total) {
    if (nf <= 0 || m <= 0 || hop < 1) return -1;
    if (variant == 0) {
        double sum = 0.0;
        for (int64_t f = 0; f < nf; ++f) {
            int64_t arg = -1;
            double best = INFINITY;
            for (int64_t j = 0; j < m; ++j)
                if (S[f * m + j] < best) { best = S[f * m + j]; arg = j; }
            ends[f] = arg;
            sum += best;
        }
        *total = sum;
        if (isinf(sum)) for (int64_t f = 0; f < nf; ++f) ends[f] = -1;
        return 0;
    }
    if (variant != 1) return -1;
    double* D = (double*)malloc(sizeof(double) * (size_t)(nf * m));
    uint8_t* match = (uint8_t*)malloc((size_t)(nf * m));
    if (!D || !match) { free(D); free(match); return -1; }
    for (int64_t f = 0; f < nf; ++f) {
        for (int64_t j = 0; j < m; ++j) {
            double skip = j >= 1 ? D[f * m + j - 1] : INFINITY;
            double prev;
            if (f == 0) prev = 0.0;
            else prev = j >= hop ? D[(f - 1) * m + j - hop] : INFINITY;
            double take = prev + S[f * m + j];
            double best = skip;
            uint8_t mt = 0;
            if (take < best) { best = take; mt = 1; }
            D[f * m + j] = best;
            match[f * m + j] = mt;
        }
    }
    *total = D[(nf - 1) * m + m - 1];
    for (int64_t f = 0; f < nf; ++f) ends[f] = -1;
    if (!isinf(*total)) {
        int64_t f = nf - 1, j = m - 1;
        while (f >= 0) {
            if (j < 0) { free(D); free(match); return -2; }
            if (match[f * m + j]) {
                ends[f] = j;
                j -= hop;
                --f;
            } else {
                --j;
            }
        }
    }
    free(D);
    free(match);
    return 0;
}
