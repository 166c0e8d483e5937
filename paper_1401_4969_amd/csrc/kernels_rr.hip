// Rayleigh-Ritz step of Algorithm 4.1 (equation (Eigen_Augment_Problem)) on
// V_0H + span{u~_1..u~_q}, solved on the device in one workgroup per problem.
//
// With the coarse generalized eigendecomposition K_H V = M_H V Lambda (V^T M_H V = I,
// computed once at setup), the border vectors a = P^T K u~, b = P^T M u~ and the
// scalars alpha = u~^T K u~, beta = u~^T M u~, the pencil on [P V, w] with the
// B-orthogonalised directions w = u~ - P V g (g = V^T b) is
//     A = [[Lambda, F], [F^T, Aw]],  B = [[I, 0], [0, Bw]],
//     F = f - Lambda g (f = V^T a),  Bw = beta - g^T g,
//     Aw = alpha - g^T f - f^T g + g^T Lambda g.
// With Bw = L L^T and Z = F L^-T, W = L^-1 Aw L^-T this is the standard symmetric
// arrowhead-type matrix T = [[Lambda, Z], [Z^T, W]] of size nH+q.  Its lowest q
// eigenvalues are found by multisection on the Sylvester inertia
//     #(eig T < mu) = #(Lambda_r < mu) + #(eig S(mu) < 0),
//     S(mu) = W - mu I - sum_r z_r z_r^T / (Lambda_r - mu),
// and its eigenvectors by inverse iteration with (T - sigma I)^-1 applied through
// the q x q Schur complement.  Cost O(nH q^2) per evaluation instead of the
// O((nH+q)^3) of a dense eigensolver.
#include "mlc_launch.h"

namespace {

constexpr int NTR = 256;
constexpr int NWR = NTR / 64;

__device__ __forceinline__ double bsum(double x, double* red) {
  x = wave_sum(x);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NWR; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ double bmin(double x, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int w = 1; w < NWR; ++w) s = fmin(s, red[w]);
  return s;
}

__device__ __forceinline__ int bmin_int(int x, int* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  int s = red[0];
#pragma unroll
  for (int w = 1; w < NWR; ++w) s = min(s, red[w]);
  return s;
}

// Number of eigenvalues of T below mu (Sylvester inertia through the Schur complement).
template <int Q>
__device__ int count_below(double mu, const double* Lam, const double* Z, int nH,
                           const double* W) {
  double S[Q][Q];
#pragma unroll
  for (int i = 0; i < Q; ++i)
#pragma unroll
    for (int j = 0; j < Q; ++j) S[i][j] = 0.0;
  int n = 0;
  for (int r = 0; r < nH; ++r) {
    double d = Lam[r] - mu;
    if (d < 0.0) ++n;
    if (d == 0.0) d = 1e-300;
    const double inv = 1.0 / d;
    double z[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) z[i] = Z[r * Q + i];
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) S[i][j] += z[i] * z[j] * inv;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      S[i][j] = W[i * Q + j] - S[i][j] - (i == j ? mu : 0.0);
      S[j][i] = S[i][j];
    }
  // LDL^T without pivoting: the count of negative pivots is the number of negative
  // eigenvalues (Sylvester); an exact zero pivot is nudged.
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    double d = S[k][k];
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++n;
#pragma unroll
    for (int i = k + 1; i < Q; ++i) {
      const double f = S[i][k] / d;
#pragma unroll
      for (int j = k + 1; j < Q; ++j) S[i][j] -= f * S[k][j];
    }
  }
  return n;
}

// Solve the small dense system A x = b (Gaussian elimination, partial pivoting).
template <int Q>
__device__ void small_solve(double (&A)[Q][Q], double (&b)[Q]) {
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    int p = k;
    for (int i = k + 1; i < Q; ++i)
      if (fabs(A[i][k]) > fabs(A[p][k])) p = i;
    if (p != k) {
      for (int j = 0; j < Q; ++j) {
        const double t = A[k][j];
        A[k][j] = A[p][j];
        A[p][j] = t;
      }
      const double t = b[k];
      b[k] = b[p];
      b[p] = t;
    }
    double d = A[k][k];
    if (d == 0.0) d = 1e-300;
    for (int i = k + 1; i < Q; ++i) {
      const double f = A[i][k] / d;
      for (int j = k; j < Q; ++j) A[i][j] -= f * A[k][j];
      b[i] -= f * b[k];
    }
  }
  for (int k = Q - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < Q; ++j) s -= A[k][j] * b[j];
    double d = A[k][k];
    if (d == 0.0) d = 1e-300;
    b[k] = s / d;
  }
}

template <int Q>
__global__ __launch_bounds__(NTR) void k_rr_solve(const ProbDev* probs, int m, int dst) {
  __shared__ double red[NWR];
  __shared__ int redi[NWR];
  __shared__ double sAlpha[Q * Q], sBeta[Q * Q];
  __shared__ double sGG[Q * Q], sGF[Q * Q], sGLG[Q * Q];
  __shared__ double sL[Q * Q], sW[Q * Q];
  __shared__ double sMu[Q], sS[Q], sT[Q];
  __shared__ double sLo, sHi;
  extern __shared__ double dyn[];
  const ProbDev& P = probs[blockIdx.x];
  if (m > P.L) return;
  const int tid = threadIdx.x;
  const int nH = P.nH;
  double* Lam = dyn;
  double* Z = dyn + nH;
  const double* f = P.fg;
  const double* g = P.fg + (int64_t)Q * nH;

  // 1. finish the fine-grid reductions in a fixed order
  {
    const int N = P.n_c << m;
    const int64_t nn = (int64_t)(N + 1) * (N + 1);
    const int nblk = (int)((nn + 255) / 256);
    const int nv = 2 * Q * Q + Q;
    for (int v = 0; v < 2 * Q * Q; ++v) {
      double s = 0.0;
      for (int b = tid; b < nblk; b += NTR) s += P.partials[(int64_t)b * nv + v];
      s = bsum(s, red);
      if (tid == 0) {
        if (v < Q * Q)
          sAlpha[v] = s;
        else
          sBeta[v - Q * Q] = s;
      }
    }
  }
  for (int r = tid; r < nH; r += NTR) Lam[r] = P.Lam[r];
  // 2. g^T g, g^T f, g^T Lambda g
  for (int i = 0; i < Q; ++i) {
    for (int j = 0; j < Q; ++j) {
      double a = 0.0, b = 0.0, c = 0.0;
      for (int r = tid; r < nH; r += NTR) {
        const double gi = g[(int64_t)i * nH + r];
        a += gi * g[(int64_t)j * nH + r];
        b += gi * f[(int64_t)j * nH + r];
        c += gi * P.Lam[r] * g[(int64_t)j * nH + r];
      }
      a = bsum(a, red);
      b = bsum(b, red);
      c = bsum(c, red);
      if (tid == 0) {
        sGG[i * Q + j] = a;
        sGF[i * Q + j] = b;
        sGLG[i * Q + j] = c;
      }
    }
  }
  __syncthreads();
  // 3. Bw = L L^T, W = L^-1 Aw L^-T
  if (tid == 0) {
    double Bw[Q][Q], Aw[Q][Q], L[Q][Q];
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j < Q; ++j) {
        Bw[i][j] = 0.5 * (sBeta[i * Q + j] + sBeta[j * Q + i]) -
                   0.5 * (sGG[i * Q + j] + sGG[j * Q + i]);
        Aw[i][j] = 0.5 * (sAlpha[i * Q + j] + sAlpha[j * Q + i]) - sGF[i * Q + j] -
                   sGF[j * Q + i] + 0.5 * (sGLG[i * Q + j] + sGLG[j * Q + i]);
        L[i][j] = 0.0;
      }
    for (int j = 0; j < Q; ++j) {
      double d = Bw[j][j];
      for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
      d = d > 1e-300 ? sqrt(d) : 1e-150;
      L[j][j] = d;
      for (int i = j + 1; i < Q; ++i) {
        double s = Bw[i][j];
        for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
        L[i][j] = s / d;
      }
    }
    // X = L^-1 Aw (forward substitution on columns), W = X L^-T = (L^-1 X^T)^T
    double X[Q][Q];
    for (int c = 0; c < Q; ++c)
      for (int i = 0; i < Q; ++i) {
        double s = Aw[i][c];
        for (int k = 0; k < i; ++k) s -= L[i][k] * X[k][c];
        X[i][c] = s / L[i][i];
      }
    double Wm[Q][Q];
    for (int rI = 0; rI < Q; ++rI)
      for (int i = 0; i < Q; ++i) {
        double s = X[rI][i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * Wm[rI][k];
        Wm[rI][i] = s / L[i][i];
      }
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j < Q; ++j) {
        sW[i * Q + j] = 0.5 * (Wm[i][j] + Wm[j][i]);
        sL[i * Q + j] = L[i][j];
      }
  }
  __syncthreads();
  // 4. z_r = L^-1 (f_r - Lambda_r g_r)
  for (int r = tid; r < nH; r += NTR) {
    double z[Q];
    for (int i = 0; i < Q; ++i) {
      double s = f[(int64_t)i * nH + r] - Lam[r] * g[(int64_t)i * nH + r];
      for (int k = 0; k < i; ++k) s -= sL[i * Q + k] * z[k];
      z[i] = s / sL[i * Q + i];
    }
    for (int i = 0; i < Q; ++i) Z[r * Q + i] = z[i];
  }
  __syncthreads();
  // 5. Gershgorin lower bound; upper bound from interlacing (mu_q <= Lambda_q)
  double lo;
  {
    double rowmin = 1e300;
    double cs[Q];
    for (int i = 0; i < Q; ++i) cs[i] = 0.0;
    for (int r = tid; r < nH; r += NTR) {
      double s = 0.0;
      for (int i = 0; i < Q; ++i) {
        const double a = fabs(Z[r * Q + i]);
        s += a;
        cs[i] += a;
      }
      rowmin = fmin(rowmin, Lam[r] - s);
    }
    lo = bmin(rowmin, red);
    for (int i = 0; i < Q; ++i) {
      const double c = bsum(cs[i], red);
      double w = sW[i * Q + i] - c;
      for (int j = 0; j < Q; ++j)
        if (j != i) w -= fabs(sW[i * Q + j]);
      lo = fmin(lo, w);
    }
  }
  const double hi0 = Lam[Q - 1] + 1e-12 * fabs(Lam[Q - 1]) + 1e-300;
  lo -= 1e-12 * fabs(lo) + 1e-300;
  // 6. multisection for each of the lowest Q eigenvalues
  for (int k = 0; k < Q; ++k) {
    if (tid == 0) {
      sLo = lo;
      sHi = hi0;
    }
    __syncthreads();
    for (int round = 0; round < 24; ++round) {
      const double a = sLo, b = sHi;
      if (b - a <= 4.0 * 2.220446049250313e-16 * fmax(fabs(a), fabs(b))) break;
      const double mu = a + (b - a) * (double)(tid + 1) / (double)(NTR + 1);
      const int c = count_below<Q>(mu, Lam, Z, nH, sW);
      const int t = bmin_int(c >= k + 1 ? tid : NTR, redi);
      __syncthreads();
      if (tid == t) sHi = mu;
      if (tid == t - 1) sLo = mu;
      if (t == NTR && tid == NTR - 1) sLo = mu;
      __syncthreads();
    }
    if (tid == 0) sMu[k] = 0.5 * (sLo + sHi);
    __syncthreads();
  }
  // 7. eigenvectors by inverse iteration on T - sigma I
  const int n = nH + Q;
  for (int k = 0; k < Q; ++k) {
    double* x = P.rr_x + (int64_t)k * n;
    const double mu = sMu[k];
    const double sigma = mu - fmax(8.0 * 2.220446049250313e-16 * fabs(mu), 1e-300);
    for (int r = tid; r < n; r += NTR) x[r] = 1.0 + 0.01 * (double)((r * 7 + k * 13) % 17);
    __syncthreads();
    for (int iter = 0; iter < 3; ++iter) {
      // S(sigma) and the reduced right-hand side, accumulated over r
      double Sp[Q][Q], rp[Q];
      for (int i = 0; i < Q; ++i) {
        rp[i] = 0.0;
        for (int j = 0; j < Q; ++j) Sp[i][j] = 0.0;
      }
      for (int r = tid; r < nH; r += NTR) {
        double d = Lam[r] - sigma;
        if (d == 0.0) d = 1e-300;
        const double inv = 1.0 / d;
        for (int i = 0; i < Q; ++i) {
          rp[i] += Z[r * Q + i] * x[r] * inv;
          for (int j = 0; j < Q; ++j) Sp[i][j] += Z[r * Q + i] * Z[r * Q + j] * inv;
        }
      }
      double A[Q][Q], bb[Q];
      for (int i = 0; i < Q; ++i) {
        bb[i] = x[nH + i] - bsum(rp[i], red);
        for (int j = 0; j < Q; ++j)
          A[i][j] = sW[i * Q + j] - (i == j ? sigma : 0.0) - bsum(Sp[i][j], red);
      }
      small_solve<Q>(A, bb);  // every thread holds the same s
      __syncthreads();
      for (int r = tid; r < nH; r += NTR) {
        double d = Lam[r] - sigma;
        if (d == 0.0) d = 1e-300;
        double s = x[r];
        for (int i = 0; i < Q; ++i) s -= Z[r * Q + i] * bb[i];
        x[r] = s / d;
      }
      if (tid < Q) x[nH + tid] = bb[tid];
      __syncthreads();
      for (int kp = 0; kp < k; ++kp) {
        const double* xp = P.rr_x + (int64_t)kp * n;
        double d = 0.0;
        for (int r = tid; r < n; r += NTR) d += x[r] * xp[r];
        d = bsum(d, red);
        for (int r = tid; r < n; r += NTR) x[r] -= d * xp[r];
        __syncthreads();
      }
      double nr = 0.0;
      for (int r = tid; r < n; r += NTR) nr += x[r] * x[r];
      nr = sqrt(bsum(nr, red));
      for (int r = tid; r < n; r += NTR) x[r] /= nr;
      __syncthreads();
    }
    // 8. back to the original basis: u_k = P V (y - g t) + u~ t, t = L^-T s
    if (tid == 0) {
      double t[Q];
      for (int i = Q - 1; i >= 0; --i) {
        double s = x[nH + i];
        for (int j = i + 1; j < Q; ++j) s -= sL[j * Q + i] * t[j];
        t[i] = s / sL[i * Q + i];
      }
      for (int i = 0; i < Q; ++i) {
        sT[i] = t[i];
        P.rr_t[k * Q + i] = t[i];
      }
      P.lam[dst * MLC_MAX_Q + k] = mu;
    }
    __syncthreads();
    for (int r = tid; r < nH; r += NTR) {
      double s = x[r];
      for (int i = 0; i < Q; ++i) s -= g[(int64_t)i * nH + r] * sT[i];
      P.rr_y[(int64_t)k * nH + r] = s;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_rr_solve(int max_q, const ProbDev* probs, int nprob, int m, int max_nH, int dst,
                           hipStream_t s) {
  const size_t shm = (size_t)max_nH * (1 + max_q) * sizeof(double);
  switch (max_q) {
#define MLC_RR_CASE(QQ)                                                                       \
  case QQ:                                                                                    \
    hipLaunchKernelGGL(k_rr_solve<QQ>, dim3(nprob), dim3(NTR), shm, s, probs, m, dst); \
    break;
    MLC_RR_CASE(1)
    MLC_RR_CASE(2)
    MLC_RR_CASE(3)
    MLC_RR_CASE(4)
    MLC_RR_CASE(5)
    MLC_RR_CASE(6)
    MLC_RR_CASE(7)
    MLC_RR_CASE(8)
#undef MLC_RR_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
