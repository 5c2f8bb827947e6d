/*
 * sgemm oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of what the
 * hierarchical-dataflow sgemm computes.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load this library; the GPU product
 * path never links, calls or imports it, and it shares no code, header, table
 * or helper with that path.
 *
 * What it follows (HPVM technical report, arXiv:1611.00860):
 *  - Sec. 5.1 names the benchmark "single-precision matrix multiplication"
 *    (Parboil sgemm), and Sec. 6.1 (listing "SGEMM in HPVM", SgemmLeaf) gives
 *    its BLAS-shaped operand list: A, lda, B, ldb, C, ldc, k, alpha, beta.
 *  - Sec. 2.3 marks A and B as `in` and C as `in out`: C is read and updated,
 *    so the node computes C <- alpha * (A B) + beta * C.
 *  - Sec. 2.1: every dynamic instance of SgemmLeaf computes different output
 *    elements, so the result is the element-wise definition below; the
 *    hierarchy (tiling) changes the evaluation order, not the value.
 *  The paper never writes the formula out, nor the storage layout; the
 *  readings taken here (row-major, no transpose; BLAS beta==0 / alpha==0
 *  conventions) are the ones listed in the design notes.
 *
 * Arithmetic: every FP32 input is widened exactly to double; products and
 * sums are IEEE double, evaluated in the order p = 0 .. k-1 for every output
 * element (i-p-j loop nest).  Build with -ffp-contract=off so no fused
 * multiply-add changes the rounding.
 *
 * Split-aware modes (for the reduced-precision variants; the paper only has
 * FP32): mode 1 rounds every A and B element to bfloat16 (round to nearest,
 * ties to even) before the exact FP64 sum; mode 2 writes each element as
 * hi + lo with hi = bf16(a), lo = bf16(a - hi) and sums
 * hi_a*hi_b + hi_a*lo_b + lo_a*hi_b in FP64 (the bf16x3 scheme of Henry,
 * Tang and Heinecke, "Leveraging the bfloat16 AI datatype for higher-precision
 * computations", ARITH 2019).  These modes separate the error a
 * representation carries by itself from the error of a kernel's FP32
 * accumulation.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_FP32 0
#define ORACLE_BF16 1
#define ORACLE_BF16X3 2

/* ------------------------------------------------------------------------ */
/* bfloat16 rounding, written from the IEEE 754 definition of round to       */
/* nearest, ties to even.  bfloat16 keeps the sign, the 8 exponent bits and  */
/* the top 7 fraction bits of an IEEE single; its values are exactly the     */
/* singles whose low 16 bits are zero.                                       */
/* ------------------------------------------------------------------------ */
static float bits_to_float(uint32_t u) {
  float f;
  memcpy(&f, &u, sizeof f);
  return f;
}
static uint32_t float_to_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, sizeof u);
  return u;
}

float oracle_bf16_round(float x) {
  uint32_t u = float_to_bits(x);
  if ((u & 0x7f800000u) == 0x7f800000u) {
    if (u & 0x007fffffu) /* NaN: stay NaN (quiet), keep the sign */
      return bits_to_float((u | 0x00400000u) & 0xffff0000u);
    return x; /* +-infinity is representable */
  }
  /* The two bfloat16 neighbours of x with the sign of x: `down` (toward
   * zero, the truncation) and `up` (one bfloat16 ulp further from zero). */
  uint32_t down = u & 0xffff0000u;
  uint32_t up = down + 0x00010000u;
  double ax = fabs((double)x);
  double adown = fabs((double)bits_to_float(down));
  double aup;
  if ((up & 0x7f800000u) == 0x7f800000u)
    aup = ldexp(1.0, 128); /* unbounded-exponent value just past the max */
  else
    aup = fabs((double)bits_to_float(up));
  double d_down = ax - adown; /* exact: both are singles */
  double d_up = aup - ax;
  if (d_down < d_up) return bits_to_float(down);
  if (d_up < d_down) return bits_to_float(up); /* may be +-inf: overflow */
  /* tie: pick the neighbour whose last kept fraction bit is zero */
  return ((down >> 16) & 1u) ? bits_to_float(up) : bits_to_float(down);
}

/* Round a whole array (used by the tests to pin the rounder). */
void oracle_bf16_round_array(const float* x, float* y, int64_t count) {
  for (int64_t t = 0; t < count; ++t) y[t] = oracle_bf16_round(x[t]);
}

/* hi/lo split of one single: hi = bf16(a), lo = bf16(a - hi).  a - hi is
 * exact in single precision (Sterbenz-type cancellation of the top bits). */
void oracle_bf16_split_array(const float* x, float* hi, float* lo,
                             int64_t count) {
  for (int64_t t = 0; t < count; ++t) {
    float h = oracle_bf16_round(x[t]);
    hi[t] = h;
    lo[t] = oracle_bf16_round(x[t] - h);
  }
}

/* ------------------------------------------------------------------------ */
/* Operand preparation per mode: widened copies of the representable parts.  */
/* ------------------------------------------------------------------------ */
typedef struct {
  double* hi; /* mode 0: the value; mode 1: bf16(value); mode 2: hi part */
  double* lo; /* mode 2 only: lo part; NULL otherwise                     */
  int64_t ld;
} operand;

static int prepare(const float* X, int64_t rows, int64_t cols, int64_t ldx,
                   int mode, operand* out) {
  out->hi = NULL;
  out->lo = NULL;
  out->ld = cols;
  size_t count = (size_t)(rows * cols);
  if (count == 0) return 0;
  out->hi = (double*)malloc(count * sizeof(double));
  if (!out->hi) return -1;
  if (mode == ORACLE_BF16X3) {
    out->lo = (double*)malloc(count * sizeof(double));
    if (!out->lo) return -1;
  }
  for (int64_t r = 0; r < rows; ++r)
    for (int64_t c = 0; c < cols; ++c) {
      float v = X[r * ldx + c];
      size_t o = (size_t)(r * cols + c);
      if (mode == ORACLE_FP32) {
        out->hi[o] = (double)v;
      } else if (mode == ORACLE_BF16) {
        out->hi[o] = (double)oracle_bf16_round(v);
      } else {
        float h = oracle_bf16_round(v);
        out->hi[o] = (double)h;
        out->lo[o] = (double)oracle_bf16_round(v - h);
      }
    }
  return 0;
}

static void release(operand* o) {
  free(o->hi);
  free(o->lo);
}

/* ------------------------------------------------------------------------ */
/* Forward: out[i][j] = alpha * sum_p A[i][p] B[p][j] + beta * C[i][j]        */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t m, n, k, r0, r1;
  double alpha, beta;
  const operand *A, *B;
  const float* C;
  int64_t ldc;
  double* out;
  int64_t ldo;
  int mode;
  int status;
} fwd_job;

static void* fwd_rows(void* arg) {
  fwd_job* j = (fwd_job*)arg;
  double* S = (double*)calloc((size_t)(j->n > 0 ? j->n : 1), sizeof(double));
  if (!S) {
    j->status = -1;
    return NULL;
  }
  for (int64_t i = j->r0; i < j->r1; ++i) {
    for (int64_t c = 0; c < j->n; ++c) S[c] = 0.0;
    if (j->alpha != 0.0) {
      for (int64_t p = 0; p < j->k; ++p) {
        double ah = j->A->hi[i * j->A->ld + p];
        const double* bh = j->B->hi + p * j->B->ld;
        if (j->mode == ORACLE_BF16X3) {
          double al = j->A->lo[i * j->A->ld + p];
          const double* bl = j->B->lo + p * j->B->ld;
          for (int64_t c = 0; c < j->n; ++c)
            S[c] += ah * bh[c] + ah * bl[c] + al * bh[c];
        } else {
          for (int64_t c = 0; c < j->n; ++c) S[c] += ah * bh[c];
        }
      }
    }
    for (int64_t c = 0; c < j->n; ++c) {
      double v = (j->alpha != 0.0) ? j->alpha * S[c] : 0.0;
      if (j->beta != 0.0) v += j->beta * (double)j->C[i * j->ldc + c];
      j->out[i * j->ldo + c] = v;
    }
  }
  free(S);
  j->status = 0;
  return NULL;
}

static int clamp_threads(int nthreads, int64_t rows) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if (rows < nthreads) nthreads = rows > 0 ? (int)rows : 1;
  return nthreads;
}

/* Returns 0 on success, -1 on bad arguments or allocation failure. */
int oracle_sgemm(int64_t m, int64_t n, int64_t k, double alpha,
                 const float* A, int64_t lda, const float* B, int64_t ldb,
                 double beta, const float* C, int64_t ldc, double* out,
                 int64_t ldo, int mode, int nthreads) {
  if (m < 0 || n < 0 || k < 0 || ldo < n) return -1;
  if (mode < ORACLE_FP32 || mode > ORACLE_BF16X3) return -1;
  if (beta != 0.0 && ldc < n) return -1;
  if (m == 0 || n == 0) return 0;
  operand Aop = {0}, Bop = {0};
  int need_ab = (alpha != 0.0 && k > 0);
  if (need_ab) {
    if (lda < k || ldb < n) return -1;
    if (prepare(A, m, k, lda, mode, &Aop) || prepare(B, k, n, ldb, mode, &Bop)) {
      release(&Aop);
      release(&Bop);
      return -1;
    }
  }
  nthreads = clamp_threads(nthreads, m);
  pthread_t tid[256];
  fwd_job jobs[256];
  int64_t per = (m + nthreads - 1) / nthreads;
  int status = 0;
  for (int t = 0; t < nthreads; ++t) {
    fwd_job* j = &jobs[t];
    j->m = m;
    j->n = n;
    j->k = need_ab ? k : 0;
    j->r0 = t * per < m ? t * per : m;
    j->r1 = (t + 1) * per < m ? (t + 1) * per : m;
    j->alpha = need_ab ? alpha : 0.0;
    j->beta = beta;
    j->A = &Aop;
    j->B = &Bop;
    j->C = C;
    j->ldc = ldc;
    j->out = out;
    j->ldo = ldo;
    j->mode = mode;
    j->status = 0;
    if (nthreads == 1) fwd_rows(j);
    else pthread_create(&tid[t], NULL, fwd_rows, j);
  }
  if (nthreads > 1)
    for (int t = 0; t < nthreads; ++t) pthread_join(tid[t], NULL);
  for (int t = 0; t < nthreads; ++t) status |= jobs[t].status;
  release(&Aop);
  release(&Bop);
  return status ? -1 : 0;
}

/* Selected output elements only, one dot product each: out[t] is element
 * (rows[t], cols[t]) of the definition above.  Lets a test check a handful
 * of entries of a product far too large for the full oracle. */
int oracle_sgemm_entries(int64_t m, int64_t n, int64_t k, double alpha,
                         const float* A, int64_t lda, const float* B,
                         int64_t ldb, double beta, const float* C, int64_t ldc,
                         int64_t count, const int64_t* rows,
                         const int64_t* cols, double* out, int mode) {
  if (m < 0 || n < 0 || k < 0) return -1;
  for (int64_t t = 0; t < count; ++t) {
    int64_t i = rows[t], c = cols[t];
    if (i < 0 || i >= m || c < 0 || c >= n) return -1;
    double s = 0.0;
    if (alpha != 0.0) {
      for (int64_t p = 0; p < k; ++p) {
        float a = A[i * lda + p], b = B[p * ldb + c];
        if (mode == ORACLE_FP32) {
          s += (double)a * (double)b;
        } else if (mode == ORACLE_BF16) {
          s += (double)oracle_bf16_round(a) * (double)oracle_bf16_round(b);
        } else {
          float ah = oracle_bf16_round(a), bh = oracle_bf16_round(b);
          double al = oracle_bf16_round(a - ah), bl = oracle_bf16_round(b - bh);
          s += (double)ah * (double)bh + (double)ah * bl + al * (double)bh;
        }
      }
    }
    double v = (alpha != 0.0) ? alpha * s : 0.0;
    if (beta != 0.0) v += beta * (double)C[i * ldc + c];
    out[t] = v;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Gradient of L = <G, C_out> with C_out = alpha*A*B + beta*C_in, in closed  */
/* form (FP64):                                                              */
/*   dA = alpha * G * B^T        (m x k)                                     */
/*   dB = alpha * A^T * G        (k x n)                                     */
/*   dalpha = sum_ij G_ij (A B)_ij                                           */
/*   dbeta  = sum_ij G_ij C_in_ij                                            */
/*   dC_in  = beta * G           (m x n)                                     */
/* Any of dA, dB, dCin, dalpha, dbeta may be NULL to skip it.                */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t m, n, k, r0, r1;
  double alpha;
  const float *A, *B, *G;
  int64_t lda, ldb, ldg;
  double* dA;     /* rows r0..r1 of dA (m x k)                     */
  double* dB;     /* private k x n partial of A^T G over rows      */
  double dalpha;  /* partial sum over rows r0..r1                  */
} grad_job;

static void* grad_rows(void* arg) {
  grad_job* j = (grad_job*)arg;
  double* S = (double*)calloc((size_t)(j->n > 0 ? j->n : 1), sizeof(double));
  j->dalpha = 0.0;
  for (int64_t i = j->r0; i < j->r1; ++i) {
    const float* Gi = j->G + i * j->ldg;
    /* dA[i][p] = alpha * sum_c G[i][c] B[p][c] */
    if (j->dA)
      for (int64_t p = 0; p < j->k; ++p) {
        double s = 0.0;
        const float* Bp = j->B + p * j->ldb;
        for (int64_t c = 0; c < j->n; ++c) s += (double)Gi[c] * (double)Bp[c];
        j->dA[i * j->k + p] = j->alpha * s;
      }
    /* (A B)[i][:] for dalpha, and the row-i term of A^T G for dB */
    for (int64_t c = 0; c < j->n; ++c) S[c] = 0.0;
    for (int64_t p = 0; p < j->k; ++p) {
      double a = (double)j->A[i * j->lda + p];
      const float* Bp = j->B + p * j->ldb;
      for (int64_t c = 0; c < j->n; ++c) S[c] += a * (double)Bp[c];
      if (j->dB) {
        double* dBp = j->dB + p * j->n;
        for (int64_t c = 0; c < j->n; ++c) dBp[c] += a * (double)Gi[c];
      }
    }
    for (int64_t c = 0; c < j->n; ++c) j->dalpha += (double)Gi[c] * S[c];
  }
  free(S);
  return NULL;
}

int oracle_sgemm_grad(int64_t m, int64_t n, int64_t k, double alpha,
                      double beta, const float* A, int64_t lda, const float* B,
                      int64_t ldb, const float* Cin, int64_t ldci,
                      const float* G, int64_t ldg, double* dA, double* dB,
                      double* dCin, double* dalpha, double* dbeta,
                      int nthreads) {
  if (m < 0 || n < 0 || k < 0) return -1;
  if (lda < k || ldb < n || ldci < n || ldg < n) return -1;
  nthreads = clamp_threads(nthreads, m);
  pthread_t tid[256];
  grad_job jobs[256];
  int64_t per = (m + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    grad_job* j = &jobs[t];
    j->m = m;
    j->n = n;
    j->k = k;
    j->r0 = t * per < m ? t * per : m;
    j->r1 = (t + 1) * per < m ? (t + 1) * per : m;
    j->alpha = alpha;
    j->A = A;
    j->B = B;
    j->G = G;
    j->lda = lda;
    j->ldb = ldb;
    j->ldg = ldg;
    j->dA = dA;
    j->dB = NULL;
    if (dB && k > 0 && n > 0) {
      j->dB = (double*)calloc((size_t)(k * n), sizeof(double));
      if (!j->dB) return -1;
    }
    if (nthreads == 1) grad_rows(j);
    else pthread_create(&tid[t], NULL, grad_rows, j);
  }
  if (nthreads > 1)
    for (int t = 0; t < nthreads; ++t) pthread_join(tid[t], NULL);
  /* dB = alpha * sum over the per-thread partials, in thread order */
  if (dB) {
    for (int64_t e = 0; e < k * n; ++e) {
      double s = 0.0;
      for (int t = 0; t < nthreads; ++t)
        if (jobs[t].dB) s += jobs[t].dB[e];
      dB[e] = alpha * s;
    }
  }
  double da = 0.0;
  for (int t = 0; t < nthreads; ++t) {
    da += jobs[t].dalpha;
    free(jobs[t].dB);
  }
  if (dalpha) *dalpha = da;
  if (dbeta) {
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i)
      for (int64_t c = 0; c < n; ++c)
        s += (double)G[i * ldg + c] * (double)Cin[i * ldci + c];
    *dbeta = s;
  }
  if (dCin)
    for (int64_t i = 0; i < m; ++i)
      for (int64_t c = 0; c < n; ++c)
        dCin[i * n + c] = beta * (double)G[i * ldg + c];
  return 0;
}

/* Selected entries of dA = alpha G B^T (which = 0) or dB = alpha A^T G
 * (which = 1): out[t] is element (rows[t], cols[t]). */
int oracle_grad_entries(int which, int64_t m, int64_t n, int64_t k,
                        double alpha, const float* A, int64_t lda,
                        const float* B, int64_t ldb, const float* G,
                        int64_t ldg, int64_t count, const int64_t* rows,
                        const int64_t* cols, double* out) {
  for (int64_t t = 0; t < count; ++t) {
    int64_t r = rows[t], c = cols[t];
    double s = 0.0;
    if (which == 0) { /* dA[r][c], r < m, c < k: sum over j < n */
      if (r < 0 || r >= m || c < 0 || c >= k) return -1;
      for (int64_t j = 0; j < n; ++j)
        s += (double)G[r * ldg + j] * (double)B[c * ldb + j];
    } else { /* dB[r][c], r < k, c < n: sum over i < m */
      if (r < 0 || r >= k || c < 0 || c >= n) return -1;
      for (int64_t i = 0; i < m; ++i)
        s += (double)A[i * lda + r] * (double)G[i * ldg + c];
    }
    out[t] = alpha * s;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* A one-to-one consumer node after the sgemm node: the pair the           */
/* MergeDependentNodes primitive of Sec. 4.1 fuses into one node.  Every   */
/* consumer instance reads the element its producer instance wrote and     */
/* writes one element (a 1-1 edge).  The paper gives no consumer for sgemm; */
/* these are the element-wise functions the fused entry point offers, each  */
/* written from its definition, in FP64:                                    */
/*   0 identity    d = v                                                    */
/*   1 relu        d = v when v > 0, else 0 (so NaN gives 0)                */
/*   2 bias        d = v + bias[j]   (bias: one FP32 value per column)      */
/*   3 bias, relu  d = relu(v + bias[j])                                    */
/*   4 clamp       d = lo when v < lo, hi when v > hi, else v (NaN stays)   */
/* X and D are m x n, row-major, leading dimension n.  Returns -1 for an    */
/* unknown op.                                                              */
/* ------------------------------------------------------------------------ */
static double relu64(double v) { return v > 0.0 ? v : 0.0; }

int oracle_consumer(int64_t m, int64_t n, const double* X, int op, const float* bias,
                    double lo, double hi, double* D) {
  if (op < 0 || op > 4) return -1;
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) {
      const double v = X[i * n + j];
      double d;
      switch (op) {
        case 1: d = relu64(v); break;
        case 2: d = v + (double)bias[j]; break;
        case 3: d = relu64(v + (double)bias[j]); break;
        case 4: d = v < lo ? lo : (v > hi ? hi : v); break;
        default: d = v; break;
      }
      D[i * n + j] = d;
    }
  return 0;
}
