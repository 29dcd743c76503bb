/*
 * wf_oracle.c -- CPU oracle for the anti-diagonal wavefront sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the tests, the smoke check and the benchmark's
 * cpu_baseline leg use it.  It shares no code with the HIP path.
 *
 * What it computes (the cell rule; the paper itself states no sweep, so the
 * rule is this project's reading, see the design notes):
 *
 *   For 0 <= i < m, 0 <= j < n, with N = (i-1, j), W = (i, j-1), NW = (i-1, j-1):
 *     N  = i == 0 ? top[j+1] : H[i-1][j]
 *     W  = j == 0 ? left[i]  : H[i][j-1]
 *     NW = i == 0 ? top[j]   : (j == 0 ? left[i-1] : H[i-1][j-1])
 *     H[i][j] = c[i][j] + op(N, W, NW)          op = min (rule 0) or max (rule 1)
 *
 *   top has n+1 entries (top[0] is the corner H[-1][-1]); left has m entries.
 *   A NULL top/left means the default boundary: corner 0, every other
 *   boundary value +inf for min and -inf for max, i.e. the predecessor does
 *   not exist.  With the default boundary H[i][j] is the min (max) over all
 *   monotone lattice paths (steps S, E, SE) from (0,0) to (i,j) of the sum of
 *   c along the path.
 *
 *   The max rule with two "engine" columns is the flow-shop recurrence whose
 *   closed form for identical rows is the streamed-time model (Eq. 2) of the
 *   paper's Section 2.2.
 *
 * Four arithmetic flavours of the same plain row-major double loop:
 *   oracle_sweep_f64: float32 inputs converted exactly, fp64 accumulation
 *   oracle_sweep_f32: the same loop in fp32 (one rounding per cell)
 *   oracle_sweep_i64: int32 inputs, exact int64 accumulation
 *   oracle_sweep_d64: float64 inputs, the loop in fp64 (one rounding per cell);
 *                     the paper's own computations are in FP64 (its Section 2
 *                     setup), FP32 being its variant (Section 3.2)
 *
 * Two more things computed on the same recurrence:
 *   oracle_dtw_f32: dynamic time warping of two sequences x (m values) and
 *     y (n values): the min rule with c[i][j] = |x[i] - y[j]|, the difference
 *     rounded once in fp32 (the absolute value is exact), then the fp32 loop.
 *     The paper has no such workload; it is a second input of the same rule.
 *   oracle_traceback_*: the path of predecessor choices from (m-1, n-1) back to
 *     the boundary through a computed grid H: at each cell the predecessor
 *     whose H value the rule selects, preferring NW, then N, then W when values
 *     are equal (the paper states no tie-break; this is the reading taken).
 *
 * Outputs: full grid H (row stride ldh) and/or the last row (n values), the
 * last column (m values); any output pointer may be NULL.  Memory use beyond
 * the outputs is two rows, so very large grids can be swept in bands with
 * explicit top/left boundaries taken from the band above.
 *
 * Return value: 0 on success, -1 on invalid arguments, -2 on allocation
 * failure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

#define ORACLE_INT_INF  ((int64_t)1 << 62)

static double op_f64(int rule, double a, double b, double c) {
  double r = a;
  if (rule == 0) { if (b < r) r = b; if (c < r) r = c; }
  else           { if (b > r) r = b; if (c > r) r = c; }
  return r;
}

static float op_f32(int rule, float a, float b, float c) {
  float r = a;
  if (rule == 0) { if (b < r) r = b; if (c < r) r = c; }
  else           { if (b > r) r = b; if (c > r) r = c; }
  return r;
}

static int64_t op_i64(int rule, int64_t a, int64_t b, int64_t c) {
  int64_t r = a;
  if (rule == 0) { if (b < r) r = b; if (c < r) r = c; }
  else           { if (b > r) r = b; if (c > r) r = c; }
  return r;
}

int oracle_sweep_f64(int rule, int64_t m, int64_t n,
                     const float* c, int64_t ldc,
                     const double* top, const double* left,
                     double* H, int64_t ldh,
                     double* last_row, double* last_col) {
  if (m < 0 || n < 0 || (rule != 0 && rule != 1) || ldc < n || (H && ldh < n)) return -1;
  if (m == 0 || n == 0) return 0;
  const double absent = rule == 0 ? INFINITY : -INFINITY;
  double* prev = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  double* cur = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  if (!prev || !cur) { free(prev); free(cur); return -2; }
  /* prev[j+1] holds H[i-1][j]; prev[0] holds H[i-1][-1]. Row -1 is the top boundary. */
  for (int64_t j = 0; j <= n; ++j) prev[j] = top ? top[j] : (j == 0 ? 0.0 : absent);
  for (int64_t i = 0; i < m; ++i) {
    cur[0] = left ? left[i] : absent;                 /* H[i][-1] */
    for (int64_t j = 0; j < n; ++j) {
      double N = prev[j + 1], W = cur[j], NW = prev[j];
      cur[j + 1] = (double)c[i * ldc + j] + op_f64(rule, N, W, NW);
    }
    if (H) for (int64_t j = 0; j < n; ++j) H[i * ldh + j] = cur[j + 1];
    if (last_col) last_col[i] = cur[n];
    double* t = prev; prev = cur; cur = t;
  }
  if (last_row) for (int64_t j = 0; j < n; ++j) last_row[j] = prev[j + 1];
  free(prev); free(cur);
  return 0;
}

int oracle_sweep_f32(int rule, int64_t m, int64_t n,
                     const float* c, int64_t ldc,
                     const float* top, const float* left,
                     float* H, int64_t ldh,
                     float* last_row, float* last_col) {
  if (m < 0 || n < 0 || (rule != 0 && rule != 1) || ldc < n || (H && ldh < n)) return -1;
  if (m == 0 || n == 0) return 0;
  const float absent = rule == 0 ? INFINITY : -INFINITY;
  float* prev = (float*)malloc(sizeof(float) * (size_t)(n + 1));
  float* cur = (float*)malloc(sizeof(float) * (size_t)(n + 1));
  if (!prev || !cur) { free(prev); free(cur); return -2; }
  for (int64_t j = 0; j <= n; ++j) prev[j] = top ? top[j] : (j == 0 ? 0.0f : absent);
  for (int64_t i = 0; i < m; ++i) {
    cur[0] = left ? left[i] : absent;
    for (int64_t j = 0; j < n; ++j) {
      float N = prev[j + 1], W = cur[j], NW = prev[j];
      volatile float s = c[i * ldc + j] + op_f32(rule, N, W, NW);  /* one fp32 rounding */
      cur[j + 1] = s;
    }
    if (H) for (int64_t j = 0; j < n; ++j) H[i * ldh + j] = cur[j + 1];
    if (last_col) last_col[i] = cur[n];
    float* t = prev; prev = cur; cur = t;
  }
  if (last_row) for (int64_t j = 0; j < n; ++j) last_row[j] = prev[j + 1];
  free(prev); free(cur);
  return 0;
}

/* Integer flavour.  A NULL boundary means "predecessor absent", represented
 * internally by +-2^62, which no reachable path sum of int32 inputs on a grid
 * below 2^30 cells per side can reach. */
int oracle_sweep_i64(int rule, int64_t m, int64_t n,
                     const int32_t* c, int64_t ldc,
                     const int64_t* top, const int64_t* left,
                     int64_t* H, int64_t ldh,
                     int64_t* last_row, int64_t* last_col) {
  if (m < 0 || n < 0 || (rule != 0 && rule != 1) || ldc < n || (H && ldh < n)) return -1;
  if (m == 0 || n == 0) return 0;
  const int64_t absent = rule == 0 ? ORACLE_INT_INF : -ORACLE_INT_INF;
  int64_t* prev = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!prev || !cur) { free(prev); free(cur); return -2; }
  for (int64_t j = 0; j <= n; ++j) prev[j] = top ? top[j] : (j == 0 ? 0 : absent);
  for (int64_t i = 0; i < m; ++i) {
    cur[0] = left ? left[i] : absent;
    for (int64_t j = 0; j < n; ++j) {
      int64_t N = prev[j + 1], W = cur[j], NW = prev[j];
      cur[j + 1] = (int64_t)c[i * ldc + j] + op_i64(rule, N, W, NW);
    }
    if (H) for (int64_t j = 0; j < n; ++j) H[i * ldh + j] = cur[j + 1];
    if (last_col) last_col[i] = cur[n];
    int64_t* t = prev; prev = cur; cur = t;
  }
  if (last_row) for (int64_t j = 0; j < n; ++j) last_row[j] = prev[j + 1];
  free(prev); free(cur);
  return 0;
}

/* fp64 inputs and arithmetic: the same loop as oracle_sweep_f64 with a double
 * cost (every cell one fp64 rounding after the exact min/max). */
int oracle_sweep_d64(int rule, int64_t m, int64_t n,
                     const double* c, int64_t ldc,
                     const double* top, const double* left,
                     double* H, int64_t ldh,
                     double* last_row, double* last_col) {
  if (m < 0 || n < 0 || (rule != 0 && rule != 1) || ldc < n || (H && ldh < n)) return -1;
  if (m == 0 || n == 0) return 0;
  const double absent = rule == 0 ? INFINITY : -INFINITY;
  double* prev = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  double* cur = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  if (!prev || !cur) { free(prev); free(cur); return -2; }
  for (int64_t j = 0; j <= n; ++j) prev[j] = top ? top[j] : (j == 0 ? 0.0 : absent);
  for (int64_t i = 0; i < m; ++i) {
    cur[0] = left ? left[i] : absent;
    for (int64_t j = 0; j < n; ++j) {
      double N = prev[j + 1], W = cur[j], NW = prev[j];
      volatile double s = c[i * ldc + j] + op_f64(rule, N, W, NW);  /* one fp64 rounding */
      cur[j + 1] = s;
    }
    if (H) for (int64_t j = 0; j < n; ++j) H[i * ldh + j] = cur[j + 1];
    if (last_col) last_col[i] = cur[n];
    double* t = prev; prev = cur; cur = t;
  }
  if (last_row) for (int64_t j = 0; j < n; ++j) last_row[j] = prev[j + 1];
  free(prev); free(cur);
  return 0;
}

/* Dynamic time warping, default boundary (corner 0, everything else +inf):
 *   D[i][j] = |x[i] - y[j]| + min(D[i-1][j], D[i][j-1], D[i-1][j-1])
 * in fp32: the difference is rounded once, its absolute value is exact, and the
 * sum is rounded once. */
int oracle_dtw_f32(int64_t m, int64_t n, const float* x, const float* y,
                   float* H, int64_t ldh, float* last_row, float* last_col) {
  if (m < 0 || n < 0 || (H && ldh < n)) return -1;
  if (m == 0 || n == 0) return 0;
  float* prev = (float*)malloc(sizeof(float) * (size_t)(n + 1));
  float* cur = (float*)malloc(sizeof(float) * (size_t)(n + 1));
  if (!prev || !cur) { free(prev); free(cur); return -2; }
  for (int64_t j = 0; j <= n; ++j) prev[j] = j == 0 ? 0.0f : INFINITY;
  for (int64_t i = 0; i < m; ++i) {
    cur[0] = INFINITY;
    for (int64_t j = 0; j < n; ++j) {
      volatile float d = x[i] - y[j];                  /* one fp32 rounding */
      float cost = fabsf(d);
      float N = prev[j + 1], W = cur[j], NW = prev[j];
      volatile float s = cost + op_f32(0, N, W, NW);   /* one fp32 rounding */
      cur[j + 1] = s;
    }
    if (H) for (int64_t j = 0; j < n; ++j) H[i * ldh + j] = cur[j + 1];
    if (last_col) last_col[i] = cur[n];
    float* t = prev; prev = cur; cur = t;
  }
  if (last_row) for (int64_t j = 0; j < n; ++j) last_row[j] = prev[j + 1];
  free(prev); free(cur);
  return 0;
}

/* Traceback.  Starting at (m-1, n-1), repeatedly take the predecessor of the
 * current cell whose value the rule selects -- the smallest for min, the
 * largest for max -- among NW (i-1, j-1), N (i-1, j) and W (i, j-1), with
 * boundary values for predecessors outside the grid (as in the sweep), and on
 * equal values the first of NW, N, W.  The walk ends when the chosen
 * predecessor lies outside the grid (row -1 or column -1).
 * path receives the visited cells as (i, j) pairs, (m-1, n-1) first, followed by
 * the outside predecessor it ended on: *len + 1 pairs, *len <= m + n - 1. */
#define TRACEBACK_BODY(T, ABSENT, ZERO)                                                    \
  if (m < 1 || n < 1 || (rule != 0 && rule != 1) || ldh < n || !path || !len) return -1;  \
  int64_t i = m - 1, j = n - 1, k = 0;                                                     \
  for (;;) {                                                                               \
    path[2 * k] = (int32_t)i;                                                              \
    path[2 * k + 1] = (int32_t)j;                                                          \
    ++k;                                                                                   \
    T vnw, vn, vw;                                                                         \
    if (i == 0) vnw = top ? top[j] : (j == 0 ? ZERO : ABSENT);                             \
    else if (j == 0) vnw = left ? left[i - 1] : ABSENT;                                    \
    else vnw = H[(i - 1) * ldh + (j - 1)];                                                 \
    vn = i == 0 ? (top ? top[j + 1] : ABSENT) : H[(i - 1) * ldh + j];                      \
    vw = j == 0 ? (left ? left[i] : ABSENT) : H[i * ldh + (j - 1)];                        \
    int di = -1, dj = -1; /* NW */                                                         \
    T best = vnw;                                                                          \
    if (rule == 0 ? vn < best : vn > best) { best = vn; di = -1; dj = 0; }                 \
    if (rule == 0 ? vw < best : vw > best) { best = vw; di = 0; dj = -1; }                 \
    i += di;                                                                               \
    j += dj;                                                                               \
    if (i < 0 || j < 0) break;                                                             \
  }                                                                                        \
  path[2 * k] = (int32_t)i;                                                                \
  path[2 * k + 1] = (int32_t)j;                                                            \
  *len = k;                                                                                \
  return 0;

int oracle_traceback_f32(int rule, int64_t m, int64_t n, const float* H, int64_t ldh,
                         const float* top, const float* left, int32_t* path, int64_t* len) {
  const float absent = rule == 0 ? INFINITY : -INFINITY;
  TRACEBACK_BODY(float, absent, 0.0f)
}

int oracle_traceback_f64(int rule, int64_t m, int64_t n, const double* H, int64_t ldh,
                         const double* top, const double* left, int32_t* path, int64_t* len) {
  const double absent = rule == 0 ? INFINITY : -INFINITY;
  TRACEBACK_BODY(double, absent, 0.0)
}

/* int32 grids (the device's integer results); absent boundary values are INT32_MAX
 * (min) and INT32_MIN + 1 (max), as the device stores them. */
int oracle_traceback_i32(int rule, int64_t m, int64_t n, const int32_t* H, int64_t ldh,
                         const int32_t* top, const int32_t* left, int32_t* path, int64_t* len) {
  const int32_t absent = rule == 0 ? INT32_MAX : INT32_MIN + 1;
  TRACEBACK_BODY(int32_t, absent, 0)
}
