// Algorithm 4.2 step 1 on the device: the full generalized eigendecomposition
//   K_H V = M_H V Lambda,  V^T M_H V = I,  Lambda ascending,
// of each problem's coarse stiffness and mass (symmetric, M_H positive definite), one
// workgroup per problem, so a batch of many problems runs in one launch and no library
// call (nor its workspace allocation) is involved.
//
//   1. Cholesky M_H = L L^T (right-looking, column by column);
//   2. C = L^-1 K_H L^-T by two forward substitutions (one thread per column), symmetrised;
//   3. cyclic Jacobi on C with the round-robin ordering: each round rotates n/2 disjoint
//      index pairs at once (Golub and Van Loan's symmetric Schur step, tan of the smaller
//      rotation angle), the rotations applied to C in 2 x 2 blocks of pair rows and pair
//      columns and accumulated in W; sweeps until no pair has |C_pq| above 1e-16
//      sqrt(|C_pp C_qq|);
//   4. Lambda = diag(C) sorted ascending, V = L^-T W (back substitution).
// C, W and L live in a scratch area of the problem (3 (n+1)^2 doubles); K_H is read from
// Kc and V written there (column-major), Lambda to Lam, 0 to info -- the layout the
// rocSOLVER path leaves.  The cost is O(n^3) per sweep on one compute unit, so the host
// sends only coarse spaces up to MLC_JACOBI_MAX_NH here.
#include "mlc_launch.h"

namespace {

constexpr int NTE = 1024;
constexpr double kJacobiRtol = 1e-16;
constexpr int kMaxSweeps = 60;

__global__ __launch_bounds__(NTE) void k_coarse_eig(const ProbDev* probs) {
  const ProbDev& P = probs[blockIdx.x];
  if (!P.eig_ws) return;  // this problem's coarse space goes to rocSOLVER
  const int n = P.nH;
  const int n2 = n + (n & 1);  // even: the round-robin pairs every index once per round
  const int h = n2 / 2;
  const int tid = threadIdx.x;
  double* L = P.eig_ws;               // n x n, row-major, lower triangle
  double* C = L + (int64_t)n * n;     // n2 x n2, row-major
  double* W = C + (int64_t)n2 * n2;   // n2 x n2, row-major
  const double* K = P.Kc;             // symmetric: row-major = column-major
  const double* M = P.Mc;
  __shared__ double s_c[MLC_JACOBI_MAX_NH / 2 + 1], s_s[MLC_JACOBI_MAX_NH / 2 + 1],
      s_t[MLC_JACOBI_MAX_NH / 2 + 1];
  __shared__ int s_p[MLC_JACOBI_MAX_NH / 2 + 1], s_q[MLC_JACOBI_MAX_NH / 2 + 1];
  __shared__ int s_changed;
  __shared__ double s_piv;

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
  // 2. X = L^-1 K (into W, row-major), then C = L^-1 X^T, symmetrised
  for (int j = tid; j < n; j += NTE)
    for (int i = 0; i < n; ++i) {
      double x = K[(int64_t)i * n + j];
      for (int k = 0; k < i; ++k) x -= L[(int64_t)i * n + k] * W[(int64_t)k * n2 + j];
      W[(int64_t)i * n2 + j] = x / L[(int64_t)i * n + i];
    }
  __syncthreads();
  for (int j = tid; j < n; j += NTE)  // column j of X^T is row j of X
    for (int i = 0; i < n; ++i) {
      double x = W[(int64_t)j * n2 + i];
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
    if (i >= n || j >= n) C[e] = 0.0;  // the padding index stays decoupled
    W[e] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();

  // 3. cyclic Jacobi, round-robin ordering
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) s_changed = 0;
    __syncthreads();
    for (int r = 0; r < n2 - 1; ++r) {
      for (int k = tid; k < h; k += NTE) {
        // slot 0 fixed, slots 1..n2-1 rotate by r; pair slot k with slot n2-1-k
        const int a = k, b = n2 - 1 - k;
        const int p0 = a == 0 ? 0 : (a - 1 + r) % (n2 - 1) + 1;
        const int q0 = (b - 1 + r) % (n2 - 1) + 1;
        const int p = min(p0, q0), q = max(p0, q0);
        const double app = C[(int64_t)p * n2 + p], aqq = C[(int64_t)q * n2 + q];
        const double apq = C[(int64_t)p * n2 + q];
        double c = 1.0, s = 0.0, t = 0.0;
        if (apq != 0.0 && fabs(apq) > kJacobiRtol * sqrt(fabs(app * aqq))) {
          const double tau = (aqq - app) / (2.0 * apq);
          t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          s_changed = 1;
        }
        s_p[k] = p;
        s_q[k] = q;
        s_c[k] = c;
        s_s[k] = s;
        s_t[k] = t;
      }
      __syncthreads();
      // C <- J^T C J on 2 x 2 blocks (pair rows k1, pair columns k2 >= k1; the mirrored
      // block is written from the same values), W <- W J
      for (int e = tid; e < h * h; e += NTE) {
        const int k1 = e / h, k2 = e % h;
        if (k2 < k1) continue;
        const int p1 = s_p[k1], q1 = s_q[k1], p2 = s_p[k2], q2 = s_q[k2];
        const double c1 = s_c[k1], sn1 = s_s[k1], c2 = s_c[k2], sn2 = s_s[k2];
        if (k1 == k2) {
          const double t = s_t[k1];
          const double apq = C[(int64_t)p1 * n2 + q1];
          C[(int64_t)p1 * n2 + p1] -= t * apq;
          C[(int64_t)q1 * n2 + q1] += t * apq;
          C[(int64_t)p1 * n2 + q1] = t != 0.0 ? 0.0 : apq;
          C[(int64_t)q1 * n2 + p1] = t != 0.0 ? 0.0 : apq;
          continue;
        }
        const double a = C[(int64_t)p1 * n2 + p2], b = C[(int64_t)p1 * n2 + q2];
        const double d = C[(int64_t)q1 * n2 + p2], f = C[(int64_t)q1 * n2 + q2];
        const double t00 = c1 * a - sn1 * d, t01 = c1 * b - sn1 * f;
        const double t10 = sn1 * a + c1 * d, t11 = sn1 * b + c1 * f;
        const double n00 = c2 * t00 - sn2 * t01, n01 = sn2 * t00 + c2 * t01;
        const double n10 = c2 * t10 - sn2 * t11, n11 = sn2 * t10 + c2 * t11;
        C[(int64_t)p1 * n2 + p2] = n00;
        C[(int64_t)p1 * n2 + q2] = n01;
        C[(int64_t)q1 * n2 + p2] = n10;
        C[(int64_t)q1 * n2 + q2] = n11;
        C[(int64_t)p2 * n2 + p1] = n00;
        C[(int64_t)q2 * n2 + p1] = n01;
        C[(int64_t)p2 * n2 + q1] = n10;
        C[(int64_t)q2 * n2 + q1] = n11;
      }
      for (int e = tid; e < n2 * h; e += NTE) {
        const int i = e / h, k = e % h;
        const int p = s_p[k], q = s_q[k];
        const double c = s_c[k], s = s_s[k];
        const double wp = W[(int64_t)i * n2 + p], wq = W[(int64_t)i * n2 + q];
        W[(int64_t)i * n2 + p] = c * wp - s * wq;
        W[(int64_t)i * n2 + q] = s * wp + c * wq;
      }
      __syncthreads();
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
  // back substitution L^T v = w for every eigenvector, one thread per column; C holds the
  // results row-major (its eigenvalues have been read)
  for (int r = tid; r < n; r += NTE) {
    const int src = s_perm[r];
    for (int i = n - 1; i >= 0; --i) {
      double v = W[(int64_t)i * n2 + src];
      for (int k = i + 1; k < n; ++k) v -= L[(int64_t)k * n + i] * C[(int64_t)k * n2 + r];
      C[(int64_t)i * n2 + r] = v / L[(int64_t)i * n + i];
    }
  }
  __syncthreads();
  double* V = P.Kc;
  for (int e = tid; e < n * n; e += NTE) {
    const int r = e / n, i = e % n;  // column r, row i
    V[e] = C[(int64_t)i * n2 + r];
  }
  if (tid == 0) *P.info = 0;
}

}  // namespace

hipError_t launch_coarse_eig(const ProbDev* probs, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_eig, dim3(nprob), dim3(NTE), 0, s, probs);
  return hipGetLastError();
}
