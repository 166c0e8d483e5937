// Algorithm 4.2 step 1 on the device: the full generalized eigendecomposition
//   K_H V = M_H V Lambda,  V^T M_H V = I,  Lambda ascending,
// of each problem's coarse stiffness and mass (symmetric, M_H positive definite), one
// workgroup per problem, so a batch of many problems runs in one launch and no library
// call (nor its workspace allocation) is involved.
//
//   1. Cholesky M_H = L L^T (right-looking, column by column);
//   2. C = L^-1 K_H L^-T by two forward substitutions (one thread per column), symmetrised
//      and padded with decoupled zero rows to n2 = a multiple of 32 (eig_padded);
//   3. block Jacobi on C: the n2 indices form nb blocks of 16, and a round pairs the blocks
//      by the round-robin ordering.  For each block pair the 32 x 32 diagonal block S is
//      staged in LDS and swept once by scalar cyclic Jacobi (round-robin pairs, Golub and
//      Van Loan's symmetric Schur step with the tan of the smaller angle; a pair rotates
//      when |S_pq| > 1e-16 sqrt(|S_pp S_qq|)), accumulating its rotations in Q (32 x 32).
//      The round's Q then act on the whole matrix in three streaming passes,
//      Y = (C Q)^T, C = Y Q (= Q^T C Q, C being symmetric) and W = W Q, each a 32-wide
//      product per row and block pair.  Sweeps (nb - 1 rounds) repeat until one applies no
//      rotation.  A pass over C and W covers 16 scalar rounds' worth of rotations, so the
//      traffic per sweep is that of about nb scalar rounds instead of n2;
//   4. Lambda = diag(C) sorted ascending, V = L^-T W (back substitution).
// L, C, W and Y live in a scratch area of the problem (eig_scratch_doubles(n)); K_H is read
// from Kc and V written there (column-major), Lambda to Lam, 0 to info -- the layout the
// rocSOLVER path leaves.  The host sends only coarse spaces up to MLC_JACOBI_MAX_NH here.
#include "mlc_launch.h"

namespace {

constexpr int NTE = 1024;
constexpr int BJ = 16;        // indices per Jacobi block
constexpr int PB = 2 * BJ;    // indices of a block pair
constexpr int QB = PB * PB;   // doubles of a staged 32 x 32 block
constexpr int kMaxPairs = eig_padded(MLC_JACOBI_MAX_NH) / PB;
constexpr double kJacobiRtol = 1e-16;
constexpr int kMaxSweeps = 60;
// dynamic LDS: the round's Q of every block pair, then the S of a group of pairs swept
// together (as many as fit)
constexpr int kLdsBlocks = 19;  // 152 KiB of 32 x 32 doubles
static_assert(kMaxPairs < kLdsBlocks, "the Q of every block pair must fit in LDS");

// Round-robin pairing of m slots (m even), round r: slot 0 fixed, slots 1..m-1 rotate;
// pair k couples slot k with slot m-1-k.  Returns the smaller slot in *p, the larger in *q.
__device__ __forceinline__ void rr_pair(int m, int r, int k, int* p, int* q) {
  const int a = k, b = m - 1 - k;
  const int p0 = a == 0 ? 0 : (a - 1 + r) % (m - 1) + 1;
  const int q0 = (b - 1 + r) % (m - 1) + 1;
  *p = min(p0, q0);
  *q = max(p0, q0);
}

// Matrix index of local index a (0..31) of the block pair (bp, bq).
__device__ __forceinline__ int pair_index(int bp, int bq, int a) {
  return a < BJ ? bp * BJ + a : bq * BJ + (a - BJ);
}

__global__ __launch_bounds__(NTE) void k_coarse_eig(const ProbDev* probs, int lds_blocks) {
  const ProbDev& P = probs[blockIdx.x];
  if (!P.eig_ws) return;  // this problem's coarse space goes to rocSOLVER
  const int n = P.nH;
  const int n2 = eig_padded(n);
  const int nb = n2 / BJ, np = nb / 2;
  const int group = min(np, lds_blocks - np);  // block pairs swept together
  const int tid = threadIdx.x;
  double* L = P.eig_ws;              // n x n, row-major, lower triangle
  double* C = L + (int64_t)n * n;    // n2 x n2, row-major
  double* W = C + (int64_t)n2 * n2;  // n2 x n2, row-major
  double* Y = W + (int64_t)n2 * n2;  // n2 x n2, row-major
  const double* K = P.Kc;            // symmetric: row-major = column-major
  const double* M = P.Mc;
  extern __shared__ double eig_lds[];
  double* Qs = eig_lds;                    // [np][32 x 32], row-major
  double* Ss = eig_lds + (int64_t)np * QB;  // [group][32 x 32]
  __shared__ double s_c[kMaxPairs * BJ], s_s[kMaxPairs * BJ], s_t[kMaxPairs * BJ];
  __shared__ int s_changed;
  __shared__ double s_piv;
  // the scalar sweep's index tables: round r's pair k is (s_pp, s_pq)[r][k], and the f-th
  // (k1, k2 >= k1) pair of pairs in row order is (s_k1, s_k2)[f] (integer divisions and a
  // search per task otherwise)
  constexpr int NBLK = BJ * (BJ + 1) / 2;
  __shared__ unsigned char s_pp[PB - 1][BJ], s_pq[PB - 1][BJ], s_k1[NBLK], s_k2[NBLK];
  for (int e = tid; e < (PB - 1) * BJ; e += NTE) {
    const int r = e / BJ, k = e % BJ;
    int p, q;
    rr_pair(PB, r, k, &p, &q);
    s_pp[r][k] = (unsigned char)p;
    s_pq[r][k] = (unsigned char)q;
  }
  for (int f = tid; f < NBLK; f += NTE) {
    int k1 = 0, rem = f;
    while (rem >= BJ - k1) {
      rem -= BJ - k1;
      ++k1;
    }
    s_k1[f] = (unsigned char)k1;
    s_k2[f] = (unsigned char)(k1 + rem);
  }

  // 1. L = chol(M)
  for (int e = tid; e < n * n; e += NTE) L[e] = M[e];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      const double d = sqrt(L[(int64_t)k * n + k]);
      L[(int64_t)k * n + k] = d;
      s_piv = 1.0 / d;
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < n; i += NTE) L[(int64_t)i * n + k] *= s_piv;
    __syncthreads();
    const int w = n - k - 1;
    for (int e = tid; e < w * w; e += NTE) {
      const int i = k + 1 + e / w, j = k + 1 + e % w;
      if (j <= i) L[(int64_t)i * n + j] -= L[(int64_t)i * n + k] * L[(int64_t)j * n + k];
    }
    __syncthreads();
  }
  // 2. X = L^-1 K (into Y, row-major), then C = L^-1 X^T, symmetrised and padded
  for (int j = tid; j < n; j += NTE)
    for (int i = 0; i < n; ++i) {
      double x = K[(int64_t)i * n + j];
      for (int k = 0; k < i; ++k) x -= L[(int64_t)i * n + k] * Y[(int64_t)k * n2 + j];
      Y[(int64_t)i * n2 + j] = x / L[(int64_t)i * n + i];
    }
  __syncthreads();
  for (int j = tid; j < n; j += NTE)  // column j of X^T is row j of X
    for (int i = 0; i < n; ++i) {
      double x = Y[(int64_t)j * n2 + i];
      for (int k = 0; k < i; ++k) x -= L[(int64_t)i * n + k] * C[(int64_t)k * n2 + j];
      C[(int64_t)i * n2 + j] = x / L[(int64_t)i * n + i];
    }
  __syncthreads();
  for (int e = tid; e < n2 * n2; e += NTE) {
    const int i = e / n2, j = e % n2;
    if (i < j && j < n) {
      const double a = 0.5 * (C[(int64_t)i * n2 + j] + C[(int64_t)j * n2 + i]);
      C[(int64_t)i * n2 + j] = a;
      C[(int64_t)j * n2 + i] = a;
    }
  }
  __syncthreads();
  for (int e = tid; e < n2 * n2; e += NTE) {
    const int i = e / n2, j = e % n2;
    if (i >= n || j >= n) C[e] = 0.0;  // the padding indices stay decoupled
    W[e] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();

  // 3. block Jacobi
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) s_changed = 0;
    __syncthreads();
    for (int br = 0; br < nb - 1; ++br) {
      // sweep the diagonal block of every block pair once, a group of pairs at a time
      for (int g0 = 0; g0 < np; g0 += group) {
        const int gn = min(group, np - g0);
        for (int e = tid; e < gn * QB; e += NTE) {
          const int g = e / QB, a = (e % QB) / PB, b = e % PB;
          int bp, bq;
          rr_pair(nb, br, g0 + g, &bp, &bq);
          const int ia = pair_index(bp, bq, a), ib = pair_index(bp, bq, b);
          Ss[e] = 0.5 * (C[(int64_t)ia * n2 + ib] + C[(int64_t)ib * n2 + ia]);
          Qs[(int64_t)(g0 + g) * QB + a * PB + b] = a == b ? 1.0 : 0.0;
        }
        __syncthreads();
        for (int r = 0; r < PB - 1; ++r) {
          for (int e = tid; e < gn * BJ; e += NTE) {
            const int g = e / BJ, k = e % BJ;
            const int p = s_pp[r][k], q = s_pq[r][k];
            const double* S = Ss + (int64_t)g * QB;
            const double app = S[p * PB + p], aqq = S[q * PB + q], apq = S[p * PB + q];
            double c = 1.0, s = 0.0, t = 0.0;
            if (apq != 0.0 && fabs(apq) > kJacobiRtol * sqrt(fabs(app * aqq))) {
              const double tau = (aqq - app) / (2.0 * apq);
              t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
              c = 1.0 / sqrt(1.0 + t * t);
              s = t * c;
              s_changed = 1;
            }
            s_c[e] = c;
            s_s[e] = s;
            s_t[e] = t;
          }
          __syncthreads();
          // S <- J^T S J on 2 x 2 blocks of pair rows k1 and pair columns k2 >= k1 (the
          // mirrored block written from the same values); Q <- Q J
          for (int e = tid; e < gn * (NBLK + PB * BJ); e += NTE) {
            const int g = e / (NBLK + PB * BJ), f = e % (NBLK + PB * BJ);
            double* S = Ss + (int64_t)g * QB;
            const double* cc = s_c + g * BJ;
            const double* ss = s_s + g * BJ;
            if (f < NBLK) {
              const int k1 = s_k1[f], k2 = s_k2[f];  // f-th pair (k1, k2 >= k1) in row order
              const int p1 = s_pp[r][k1], q1 = s_pq[r][k1], p2 = s_pp[r][k2], q2 = s_pq[r][k2];
              const double c1 = cc[k1], sn1 = ss[k1];
              if (k1 == k2) {
                const double t = s_t[g * BJ + k1];
                const double apq = S[p1 * PB + q1];
                S[p1 * PB + p1] -= t * apq;
                S[q1 * PB + q1] += t * apq;
                S[p1 * PB + q1] = t != 0.0 ? 0.0 : apq;
                S[q1 * PB + p1] = t != 0.0 ? 0.0 : apq;
                continue;
              }
              const double c2 = cc[k2], sn2 = ss[k2];
              const double a = S[p1 * PB + p2], b = S[p1 * PB + q2];
              const double d = S[q1 * PB + p2], h = S[q1 * PB + q2];
              const double t00 = c1 * a - sn1 * d, t01 = c1 * b - sn1 * h;
              const double t10 = sn1 * a + c1 * d, t11 = sn1 * b + c1 * h;
              const double n00 = c2 * t00 - sn2 * t01, n01 = sn2 * t00 + c2 * t01;
              const double n10 = c2 * t10 - sn2 * t11, n11 = sn2 * t10 + c2 * t11;
              S[p1 * PB + p2] = n00;
              S[p1 * PB + q2] = n01;
              S[q1 * PB + p2] = n10;
              S[q1 * PB + q2] = n11;
              S[p2 * PB + p1] = n00;
              S[q2 * PB + p1] = n01;
              S[p2 * PB + q1] = n10;
              S[q2 * PB + q1] = n11;
            } else {
              const int i = (f - NBLK) / BJ, k = (f - NBLK) % BJ;
              const int p = s_pp[r][k], q = s_pq[r][k];
              double* Q = Qs + (int64_t)(g0 + g) * QB;
              const double c = cc[k], s = ss[k];
              const double wp = Q[i * PB + p], wq = Q[i * PB + q];
              Q[i * PB + p] = c * wp - s * wq;
              Q[i * PB + q] = s * wp + c * wq;
            }
          }
          __syncthreads();
        }
      }
      // apply the round's rotations: Y = (C Q)^T and W = W Q, then C = Y Q.  A task is one
      // row and one block pair: 32 values in, 32 out (lanes take consecutive rows)
      for (int pass = 0; pass < 2; ++pass) {
        for (int task = tid; task < 2 * np * n2; task += NTE) {
          const int which = task / (np * n2);  // pass 0: 0 = C -> Y^T, 1 = W; pass 1: C = Y Q
          if (pass == 1 && which == 1) break;
          const int k = (task % (np * n2)) / n2, i = task % n2;
          int bp, bq;
          rr_pair(nb, br, k, &bp, &bq);
          const double* src = pass == 1 ? Y : (which == 0 ? C : W);
          double* dst = pass == 1 ? C : W;
          const double* Q = Qs + (int64_t)k * QB;
          double v[PB];
#pragma unroll
          for (int a = 0; a < PB; ++a) v[a] = src[(int64_t)i * n2 + pair_index(bp, bq, a)];
#pragma unroll 4
          for (int j = 0; j < PB; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < PB; ++a) acc += v[a] * Q[a * PB + j];
            const int ij = pair_index(bp, bq, j);
            if (pass == 0 && which == 0)
              Y[(int64_t)ij * n2 + i] = acc;
            else
              dst[(int64_t)i * n2 + ij] = acc;
          }
        }
        __syncthreads();
      }
    }
    if (s_changed == 0) break;
    __syncthreads();
  }

  // 4. Lambda ascending (ties by index); V = L^-T W, column-major into Kc
  __shared__ int s_perm[MLC_JACOBI_MAX_NH];
  for (int i = tid; i < n; i += NTE) {
    const double di = C[(int64_t)i * n2 + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = C[(int64_t)j * n2 + j];
      rank += (dj < di || (dj == di && j < i)) ? 1 : 0;
    }
    s_perm[rank] = i;
    P.Lam[rank] = di;
  }
  __syncthreads();
  // back substitution L^T v = w for every eigenvector, one thread per column; Y holds the
  // results row-major
  for (int r = tid; r < n; r += NTE) {
    const int src = s_perm[r];
    for (int i = n - 1; i >= 0; --i) {
      double v = W[(int64_t)i * n2 + src];
      for (int k = i + 1; k < n; ++k) v -= L[(int64_t)k * n + i] * Y[(int64_t)k * n2 + r];
      Y[(int64_t)i * n2 + r] = v / L[(int64_t)i * n + i];
    }
  }
  __syncthreads();
  double* V = P.Kc;
  for (int e = tid; e < n * n; e += NTE) {
    const int r = e / n, i = e % n;  // column r, row i
    V[e] = Y[(int64_t)i * n2 + r];
  }
  if (tid == 0) *P.info = 0;
}

}  // namespace

hipError_t launch_coarse_eig(const ProbDev* probs, int nprob, hipStream_t s) {
  const size_t lds = (size_t)kLdsBlocks * QB * sizeof(double);
  hipLaunchKernelGGL(k_coarse_eig, dim3(nprob), dim3(NTE), lds, s, probs, kLdsBlocks);
  return hipGetLastError();
}
