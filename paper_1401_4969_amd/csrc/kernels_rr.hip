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
//
// One workgroup of 1024 (q <= 2) or 512 threads per problem (many waves hide the latency
// of the short loops).  Reductions are batched: each wave reduces its partial sums across lanes (DPP
// moves) and writes them to LDS, and one barrier later every value is summed over the
// waves in a fixed order (deterministic).  Multisection evaluates G points per round, GS
// consecutive lanes per point (about 32 terms each), reduced by DPP inside the wave; wave
// k then updates bracket k from all points (one per lane: DPP extremes, a ballot for the
// first point attaining each) and places its next points.  The inverse-iteration vectors
// live in LDS.
#include "mlc_launch.h"

namespace {

// Workgroup size: 1024 threads for q <= 2; 512 above, where the q(q+1)/2 accumulators of
// a point need more than the 128 registers a 1024-thread workgroup allows.
template <int Q>
constexpr int rr_threads() { return Q <= 2 ? 1024 : 512; }

// Wave-reduce x and park it in lds[wave * stride + v]; the caller barriers, then sums.
// wave_sum of K values, step by step over all of them (the K dependent chains of cross-lane
// moves interleave instead of running one after another); bitwise equal to K wave_sums.
template <int K>
__device__ __forceinline__ void wave_sum_n(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = v[k] + dpp_f64<0xb1, 0xf>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = v[k] + dpp_f64<0x4e, 0xf>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = v[k] + dpp_f64<0x114, 0xf>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = v[k] + dpp_f64<0x118, 0xf>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = v[k] + dpp_f64<0x142, 0xa>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = v[k] + dpp_f64<0x143, 0xc>(v[k], 0.0);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = read_lane_f64(v[k], 63);
}

__device__ __forceinline__ void park(double x, int v, double* lds, int stride) {
  x = wave_sum(x);
  if ((threadIdx.x & 63) == 0) lds[(threadIdx.x >> 6) * stride + v] = x;
}

template <int NW>
__device__ __forceinline__ double gather(int v, const double* lds, int stride) {
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += lds[w * stride + v];
  return s;
}

// Packed lower triangle of a symmetric QxQ matrix: entry (i, j), j <= i, at tri(i, j).
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Number of negative eigenvalues of a symmetric QxQ matrix given by its packed lower
// triangle (LDL^T, Sylvester); an exact zero pivot is nudged.  det receives the product
// of the pivots (the determinant).  Indices are compile-time constants, so the matrix
// stays in registers.
template <int Q>
__device__ int neg_inertia(double (&S)[Q * (Q + 1) / 2], double& det) {
  int n = 0;
  det = 1.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    double d = S[tri(k, k)];
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++n;
    det *= d;
#pragma unroll
    for (int i = k + 1; i < Q; ++i) {
      const double f = S[tri(i, k)] / d;
#pragma unroll
      for (int j = k + 1; j <= i; ++j) S[tri(i, j)] -= f * S[tri(j, k)];
    }
  }
  return n;
}

// LU factorisation with partial pivoting of a QxQ matrix held in registers (indices are
// compile-time constants and row exchanges are selects, so nothing leaves registers):
// piv[k] is the row exchanged with row k at step k, the multipliers of step k are left in
// column k below the diagonal, U above; an exact zero pivot is nudged.
template <int Q>
__device__ __forceinline__ void lu_factor(double (&A)[Q][Q], int (&piv)[Q]) {
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    int p = k;
    double best = fabs(A[k][k]);
#pragma unroll
    for (int i = k + 1; i < Q; ++i)
      if (fabs(A[i][k]) > best) {
        best = fabs(A[i][k]);
        p = i;
      }
    piv[k] = p;
#pragma unroll
    for (int i = k + 1; i < Q; ++i) {
      const bool sw = i == p;
#pragma unroll
      for (int j = k; j < Q; ++j) {
        const double t = A[k][j];
        A[k][j] = sw ? A[i][j] : t;
        A[i][j] = sw ? t : A[i][j];
      }
    }
    double d = A[k][k];
    if (d == 0.0) d = 1e-300;
    A[k][k] = d;
#pragma unroll
    for (int i = k + 1; i < Q; ++i) {
      const double f = A[i][k] / d;
      A[i][k] = f;
#pragma unroll
      for (int j = k + 1; j < Q; ++j) A[i][j] -= f * A[k][j];
    }
  }
}

// Solve with the factors of lu_factor: the exchanges and eliminations replayed on b in
// the order of the factorisation, then back substitution; x returned in b.
template <int Q>
__device__ __forceinline__ void lu_solve(const double (&A)[Q][Q], const int (&piv)[Q],
                                         double (&b)[Q]) {
#pragma unroll
  for (int k = 0; k < Q; ++k) {
#pragma unroll
    for (int i = k + 1; i < Q; ++i) {
      const bool sw = i == piv[k];
      const double t = b[k];
      b[k] = sw ? b[i] : t;
      b[i] = sw ? t : b[i];
    }
#pragma unroll
    for (int i = k + 1; i < Q; ++i) b[i] -= A[i][k] * b[k];
  }
#pragma unroll
  for (int k = Q - 1; k >= 0; --k) {
    double s = b[k];
#pragma unroll
    for (int j = k + 1; j < Q; ++j) s -= A[k][j] * b[j];
    b[k] = s / A[k][k];
  }
}

// Lanes per multisection point: the largest power of two up to 64 that leaves at least
// `points` points per round.
constexpr int rr_group_lanes(int ntr, int points) {
  int gs = 64;
  while (gs > 1 && ntr / gs < points) gs >>= 1;
  return gs;
}

// Offsets of a round's points from a centre, as fractions of a scale: the centre itself
// (for an odd count) and pairs +-s on a geometric ladder from hi down to lo.  Guided rounds
// use the bracket width and 3e-2 ... 1e-6; the first round uses the predicted level change
// and 0.2 ... 0.02.
__device__ inline double ladder_offset(int j, int per_bracket, double hi, double lo) {
  const int odd = per_bracket & 1, pairs = per_bracket / 2;
  if (j < odd) return 0.0;
  const int i = (j - odd) >> 1;
  const double s = pairs == 1 ? sqrt(hi * lo) : hi * pow(lo / hi, (double)i / (double)(pairs - 1));
  return ((j - odd) & 1) ? s : -s;
}

// Dynamic LDS of k_rr_solve in doubles: Lambda, Z, f, g and the q eigenvectors.
__host__ __device__ inline size_t rr_dyn_doubles(int nH, int q) {
  return (size_t)nH * (1 + 3 * q) + (size_t)q * (nH + q);
}

template <int Q>
__global__ __launch_bounds__(rr_threads<Q>()) void k_rr_solve(const ProbDev* probs, int m, int dst) {
  constexpr int NTR = rr_threads<Q>();
  constexpr int NWR = NTR / 64;
  constexpr int NV = 3 * Q * Q + Q + 1;
  __shared__ double park_lds[NWR * NV];
  __shared__ double vals[NV];
  __shared__ double sAlpha[Q * Q], sBeta[Q * Q];
  __shared__ double sL[Q * Q], sW[Q * Q];
  __shared__ double sMu[Q], sT[Q];
  __shared__ double sBw[Q * Q], sAw[Q * Q], sX[Q * Q], sWm[Q * Q];  // one-thread work arrays
  extern __shared__ double dyn[];
  const ProbDev& P = probs[blockIdx.x];
  if (m > P.L) return;
  const int tid = threadIdx.x;
  const int nH = P.nH;
  double* Lam = dyn;                 // nH
  double* Z = dyn + nH;              // nH * Q
  double* f = dyn + nH * (1 + Q);    // Q * nH
  double* g = f + Q * nH;            // Q * nH
  double* X = g + Q * nH;            // Q * (nH + Q): eigenvectors of the reduced problem

  // 1. finish the fine-grid reductions (alpha, beta) in a fixed order; stage the
  //    coarse quantities in LDS
  {
    const int N = P.n_c << (m + P.order - 1);  // grid of the level's element nodes
    const int64_t nn = (int64_t)(N + 1) * (N + 1);
    const int nblk = (int)((nn + 255) / 256);
    const int nvp = 2 * Q * Q + Q;
    constexpr int NAB = 2 * Q * Q;
    if constexpr (NAB <= 32) {
      // one pass over the block partials for every value, then every wave sum before one
      // store per wave (a store after each sum would serialise them)
      double sv[NAB];
#pragma unroll
      for (int u = 0; u < NAB; ++u) sv[u] = 0.0;
      for (int b = tid; b < nblk; b += NTR) {
        const double* pb = P.partials + (int64_t)b * nvp;
#pragma unroll
        for (int u = 0; u < NAB; ++u) sv[u] += pb[u];
      }
      wave_sum_n(sv);
      if ((tid & 63) == 0) {
#pragma unroll
        for (int u = 0; u < NAB; ++u) park_lds[(tid >> 6) * NV + u] = sv[u];
      }
    } else {
      // one pass over the block partials per group of 8 values (independent loads)
      for (int v0 = 0; v0 < NAB; v0 += 8) {
        double sv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) sv[u] = 0.0;
        for (int b = tid; b < nblk; b += NTR) {
          const double* pb = P.partials + (int64_t)b * nvp + v0;
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (v0 + u < NAB) sv[u] += pb[u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (v0 + u < NAB) park(sv[u], v0 + u, park_lds, NV);
      }
    }
    for (int r = tid; r < nH; r += NTR) Lam[r] = P.Lam[r];
    for (int e = tid; e < 2 * Q * nH; e += NTR) f[e] = P.fg[e];
    __syncthreads();
    for (int v = tid; v < 2 * Q * Q; v += NTR) {
      const double s = gather<NWR>(v, park_lds, NV);
      if (v < Q * Q)
        sAlpha[v] = s;
      else
        sBeta[v - Q * Q] = s;
      if (Q == 1) P.rr_ab[v] = s;
    }
    __syncthreads();
  }
  // 2. g^T g, g^T f, g^T Lambda g (one batched reduction)
  if constexpr (3 * Q * Q <= 32) {  // every product in one pass, the wave sums before one store
    double acc[3 * Q * Q];
#pragma unroll
    for (int e = 0; e < 3 * Q * Q; ++e) acc[e] = 0.0;
    for (int r = tid; r < nH; r += NTR) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double gi = g[i * nH + r];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          acc[i * Q + j] += gi * g[j * nH + r];
          acc[Q * Q + i * Q + j] += gi * f[j * nH + r];
          acc[2 * Q * Q + i * Q + j] += gi * Lam[r] * g[j * nH + r];
        }
      }
    }
    wave_sum_n(acc);
    if ((tid & 63) == 0) {
#pragma unroll
      for (int e = 0; e < 3 * Q * Q; ++e) park_lds[(tid >> 6) * NV + e] = acc[e];
    }
  } else {
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j < Q; ++j) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int r = tid; r < nH; r += NTR) {
          const double gi = g[i * nH + r];
          a += gi * g[j * nH + r];
          b += gi * f[j * nH + r];
          c += gi * Lam[r] * g[j * nH + r];
        }
        park(a, i * Q + j, park_lds, NV);
        park(b, Q * Q + i * Q + j, park_lds, NV);
        park(c, 2 * Q * Q + i * Q + j, park_lds, NV);
      }
  }
  __syncthreads();
  for (int v = tid; v < 3 * Q * Q; v += NTR) vals[v] = gather<NWR>(v, park_lds, NV);
  __syncthreads();
  // 3. Bw = L L^T, W = L^-1 Aw L^-T (one thread; Q <= 8)
  if (tid == 0) {  // LDS work arrays: Bw, Aw, L (sL), X = L^-1 Aw, Wm = X L^-T
    const double* GG = vals;
    const double* GF = vals + Q * Q;
    const double* GLG = vals + 2 * Q * Q;
    double* Bw = sBw;
    double* Aw = sAw;
    double* L = sL;
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j < Q; ++j) {
        Bw[i * Q + j] = 0.5 * (sBeta[i * Q + j] + sBeta[j * Q + i]) - 0.5 * (GG[i * Q + j] + GG[j * Q + i]);
        Aw[i * Q + j] = 0.5 * (sAlpha[i * Q + j] + sAlpha[j * Q + i]) - GF[i * Q + j] - GF[j * Q + i] +
                        0.5 * (GLG[i * Q + j] + GLG[j * Q + i]);
        L[i * Q + j] = 0.0;
      }
    for (int j = 0; j < Q; ++j) {
      double d = Bw[j * Q + j];
      for (int k = 0; k < j; ++k) d -= L[j * Q + k] * L[j * Q + k];
      d = d > 1e-300 ? sqrt(d) : 1e-150;
      L[j * Q + j] = d;
      for (int i = j + 1; i < Q; ++i) {
        double s = Bw[i * Q + j];
        for (int k = 0; k < j; ++k) s -= L[i * Q + k] * L[j * Q + k];
        L[i * Q + j] = s / d;
      }
    }
    double* X = sX;
    for (int c = 0; c < Q; ++c)
      for (int i = 0; i < Q; ++i) {
        double s = Aw[i * Q + c];
        for (int k = 0; k < i; ++k) s -= L[i * Q + k] * X[k * Q + c];
        X[i * Q + c] = s / L[i * Q + i];
      }
    double* Wm = sWm;
    for (int rI = 0; rI < Q; ++rI)
      for (int i = 0; i < Q; ++i) {
        double s = X[rI * Q + i];
        for (int k = 0; k < i; ++k) s -= L[i * Q + k] * Wm[rI * Q + k];
        Wm[rI * Q + i] = s / L[i * Q + i];
      }
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j < Q; ++j) sW[i * Q + j] = 0.5 * (Wm[i * Q + j] + Wm[j * Q + i]);
  }
  __syncthreads();
  // 4. z_r = L^-1 (f_r - Lambda_r g_r)
  for (int r = tid; r < nH; r += NTR) {
    double z[Q];
    for (int i = 0; i < Q; ++i) {
      double s = f[i * nH + r] - Lam[r] * g[i * nH + r];
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
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) rowmin = fmin(rowmin, __shfl_xor(rowmin, o, 64));
    for (int i = 0; i < Q; ++i) park(cs[i], i, park_lds, NV);
    if ((tid & 63) == 0) park_lds[(tid >> 6) * NV + Q] = rowmin;
    __syncthreads();
    lo = park_lds[Q];
    for (int w = 1; w < NWR; ++w) lo = fmin(lo, park_lds[w * NV + Q]);
    for (int i = 0; i < Q; ++i) {
      double w = sW[i * Q + i] - gather<NWR>(i, park_lds, NV);
      for (int j = 0; j < Q; ++j)
        if (j != i) w -= fabs(sW[i * Q + j]);
      lo = fmin(lo, w);
    }
    __syncthreads();
  }
  lo -= 1e-12 * fabs(lo) + 1e-300;
  // 6. multisection for all q eigenvalues at once: each round evaluates G points over the
  //    q brackets (G/q per bracket, GS lanes per point; the work of a round grows with G
  //    while the rounds fall only with log G, so G is kept small: 16 points, 32 for
  //    q >= 5, at least 2 per bracket); every point's inertia count c tightens every bracket: mu is an upper
  //    bound of eigenvalue k when c >= k + 1 and a lower bound when c <= k.  Upper bounds
  //    start from interlacing (mu_k <= Lambda_k).
  //    A bracket's points are spread uniformly until it holds exactly one eigenvalue and no
  //    pole (the inertia counts at its ends differ by one and the numbers of Lambda_r below
  //    them agree): det S(mu) is then smooth on the bracket and changes sign once, at the
  //    eigenvalue, and the next round centres the bracket's points on the regula falsi
  //    estimate from det S at the two ends, or from an inverse quadratic through the two
  //    ends and the nearest point of the round outside the bracket (same pole count), when
  //    that estimate falls inside.  A guided round that shrinks its bracket by less than 4x
  //    is followed by a uniform one.  The first round places a bracket's points around a
  //    prediction of the eigenvalue: the discrete eigenvalues approach their limit as h^2
  //    (Section 3), so with Lambda_k the coarse one (level 0) and lambda_k the previous
  //    level's, the model lambda_l = lambda* + C 4^-l gives the change of level m as
  //    3 C 4^-m with C = (Lambda_k - lambda_k) / (1 - 4^(1-m)), and the points sit at the
  //    predicted value +-(0.2 ... 0.02) of that change (level 1 has no such model: there
  //    they sit below lambda_k at 1e-1 down to 1e-6 of it).  Where the points go changes
  //    only how fast the brackets shrink, never what they contain.
  // 16 points per round, 32 from q = 5 on (Example 6.2, q = 6: 2 points a bracket needed
  // so many rounds that doubling the points gained 36 us per step; at q = 3 it lost 27 us)
  constexpr int GS = rr_group_lanes(NTR, Q >= 5 ? 32 : 16);
  constexpr int G = NTR / GS;  // >= 2 Q, <= 64
  constexpr int GQ = G / Q;    // points per bracket, >= 2
  const int pnt = tid / GS, gl = tid % GS;
  const int kb = pnt / GQ, j = pnt % GQ;  // this point's bracket and position
  const bool active = kb < Q;
  const int kk = active ? kb : 0;
  const double off = ladder_offset(j, GQ, 3e-2, 1e-6);
  const double frac = (double)(j + 1) / (double)(GQ + 1);  // uniform position
  __shared__ double sA[Q], sB[Q], sFA[Q], sFB[Q], sEst[Q], ptMu[G], ptDet[G];
  __shared__ int sCA[Q], sCB[Q], sNA[Q], sNB[Q], sGuide[Q], ptCnt[G], ptLess[G];
  __shared__ double ptWarm[G];  // first-round points (in LDS: kept out of the loop's registers)
  if (gl == 0) {
    const double prevk = P.lam[(1 - dst) * MLC_MAX_Q + kk];
    double warm = prevk * (1.0 - 1e-1 * pow(1e-5, (double)j / (double)(GQ - 1)));
    if (m >= 2 && Lam[kk] > prevk) {
      const double dl = (Lam[kk] - prevk) * (3.0 * ldexp(1.0, -2 * m) / (1.0 - ldexp(1.0, 2 - 2 * m)));
      warm = prevk - dl + dl * ladder_offset(j, GQ, 0.2, 0.02);
    }
    ptWarm[pnt] = warm;
  }
  if (tid < Q) {
    sA[tid] = lo;
    sB[tid] = Lam[tid] + 1e-12 * fabs(Lam[tid]) + 1e-300;
    sFA[tid] = sFB[tid] = sEst[tid] = 0.0;
    sCA[tid] = sCB[tid] = -1;  // ends not evaluated yet
    sNA[tid] = sNB[tid] = 0;
    sGuide[tid] = 0;
  }
  __syncthreads();
  for (int round = 0; round < 200; ++round) {
    const double a = sA[kk], bnd = sB[kk];
    double mu = a + (bnd - a) * frac;
    if (round == 0) {
      const double warm = ptWarm[pnt];
      if (warm > a && warm < bnd) mu = warm;
    } else if (sGuide[kk]) {
      const double gm = sEst[kk] + off * (bnd - a);
      mu = (gm > a && gm < bnd) ? gm : a + 0.5 * (bnd - a);
    }
    double S[Q * (Q + 1) / 2];  // packed lower triangle
#pragma unroll
    for (int e = 0; e < Q * (Q + 1) / 2; ++e) S[e] = 0.0;
    double nless = 0.0;
    for (int r = gl; r < nH; r += GS) {
      double d = Lam[r] - mu;
      if (d < 0.0) nless += 1.0;
      if (d == 0.0) d = 1e-300;
      const double inv = 1.0 / d;
      double z[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) z[i] = Z[r * Q + i];
#pragma unroll
      for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int jj = 0; jj <= i; ++jj) S[tri(i, jj)] += z[i] * z[jj] * inv;
    }
    nless = group_sum_last(nless, GS);
#pragma unroll
    for (int e = 0; e < Q * (Q + 1) / 2; ++e) S[e] = group_sum_last(S[e], GS);
    if (gl == GS - 1) {  // the group's sums are complete in its last lane
#pragma unroll
      for (int i = 0; i < Q; ++i)
#pragma unroll
        for (int jj = 0; jj <= i; ++jj)
          S[tri(i, jj)] = sW[i * Q + jj] - S[tri(i, jj)] - (i == jj ? mu : 0.0);
      double det;
      const int neg = neg_inertia<Q>(S, det);
      ptMu[pnt] = mu;
      ptDet[pnt] = det;
      ptLess[pnt] = (int)nless;
      ptCnt[pnt] = active ? (int)nless + neg : -1;
    }
    __syncthreads();
    if ((tid >> 6) < Q) {  // wave k tightens bracket k from every point (lane p: point p)
      const int k = tid >> 6, ln = tid & 63;
      const double inf = __builtin_inf();
      const int cp = ln < G ? ptCnt[ln] : -1;
      const double mp = ln < G ? ptMu[ln] : 0.0;
      const int lp = ln < G ? ptLess[ln] : -1;
      const bool up = cp >= k + 1, down = cp >= 0 && cp <= k;
      // the highest lower and the lowest upper point, each the first such point in order
      const auto mx = [](double x, double y) { return fmax(x, y); };
      const auto mn = [](double x, double y) { return fmin(x, y); };
      double lo2 = group_reduce_last(down ? mp : -inf, 64, -inf, mx);
      double hi2 = group_reduce_last(up ? mp : inf, 64, inf, mn);
      lo2 = read_lane_f64(lo2, 63);
      hi2 = read_lane_f64(hi2, 63);
      const unsigned long long bl = __ballot(down && mp == lo2), bh = __ballot(up && mp == hi2);
      // the new ends (every lane: the third point below needs them)
      const double a0 = sA[k], b0 = sB[k];
      const int ia = (bl != 0ull && lo2 > a0) ? __ffsll(bl) - 1 : -1;  // the points that
      const int ib = (bh != 0ull && hi2 < b0) ? __ffsll(bh) - 1 : -1;  // become the ends
      const double ak = ia >= 0 ? lo2 : a0, bk = ib >= 0 ? hi2 : b0;
      const int na = ia >= 0 ? ptLess[ia] : sNA[k], nb = ib >= 0 ? ptLess[ib] : sNB[k];
      // the point of this round nearest the new bracket from outside, with its pole count
      const bool outside = cp >= 0 && lp == na && (mp < ak || mp > bk);
      double dn = group_reduce_last(outside ? (mp < ak ? ak - mp : mp - bk) : inf, 64, inf, mn);
      dn = read_lane_f64(dn, 63);
      const unsigned long long bn = __ballot(outside && (mp < ak ? ak - mp : mp - bk) == dn);
      if (ln == 0) {
        double fa = sFA[k], fb = sFB[k];
        int ca = sCA[k], cb = sCB[k];
        if (ia >= 0) {
          fa = ptDet[ia];
          ca = ptCnt[ia];
        }
        if (ib >= 0) {
          fb = ptDet[ib];
          cb = ptCnt[ib];
        }
        const bool isolated = cb - ca == 1 && na == nb && fa != 0.0 && fb != 0.0 &&
                              (fa < 0.0) != (fb < 0.0) && isfinite(fa) && isfinite(fb);
        const bool slow = sGuide[k] && bk - ak > 0.25 * (b0 - a0);
        double est = ak;
        if (isolated) {
          est = ak + (bk - ak) * (fa / (fa - fb));  // regula falsi
          if (bn != 0ull) {  // inverse quadratic through (ak, fa), (bk, fb), (x2, f2)
            const int i2 = __ffsll(bn) - 1;
            const double x2 = ptMu[i2];
            // scaled by a power of two (exact) so that the cubic products stay in range
            const int ex = ilogb(fmax(fabs(fa), fmax(fabs(fb), fabs(ptDet[i2]))));
            const double f0 = ldexp(fa, -ex), f1 = ldexp(fb, -ex), f2 = ldexp(ptDet[i2], -ex);
            if (f2 != f0 && f2 != f1 && isfinite(f2)) {  // Lagrange weights over one denominator
              const double e = ak + ((bk - ak) * (f0 * f2 * (f2 - f0)) - (x2 - ak) * (f0 * f1 * (f1 - f0))) /
                                        ((f1 - f0) * (f1 - f2) * (f2 - f0));
              if (e > ak && e < bk) est = e;
            }
          }
        }
        sA[k] = ak;
        sB[k] = bk;
        sFA[k] = fa;
        sFB[k] = fb;
        sCA[k] = ca;
        sCB[k] = cb;
        sNA[k] = na;
        sNB[k] = nb;
        sGuide[k] = isolated && !slow;
        sEst[k] = est;
      }
    }
    __syncthreads();
    bool done = true;
#pragma unroll
    for (int k = 0; k < Q; ++k)
      if (sB[k] - sA[k] > 4.0 * 2.220446049250313e-16 * fmax(fabs(sA[k]), fabs(sB[k]))) done = false;
    if (done) break;
  }
  if (tid < Q) sMu[tid] = 0.5 * (sA[tid] + sB[tid]);
  __syncthreads();
  // 7. eigenvectors by inverse iteration on T - sigma I (two steps), classical
  //    Gram-Schmidt against the previous ones.  Every entry of a vector is read and
  //    written by one thread only (entries tid, tid + NTR, ...), so only the reductions
  //    of a step need barriers, and every thread solves the q x q Schur system itself, in
  //    registers.  The Schur matrix W - sigma I - sum_r z_r z_r^T / (Lambda_r - sigma)
  //    depends on sigma only: it is summed and factored in the first step and the factors
  //    are reused in the second.  Reduction slots: Schur sums at 0 .. Q + Q^2 - 1,
  //    Gram-Schmidt products after them, the norm last, so no slot is rewritten while
  //    another wave may still read it.
  const int n = nH + Q;
  const int lane = tid & 63, wv = tid >> 6;
  constexpr int GS_SLOT = Q + Q * Q, NORM_SLOT = GS_SLOT + Q;
  for (int k = 0; k < Q; ++k) {
    double* x = X + k * n;
    const double mu = sMu[k];
    const double sigma = mu - fmax(8.0 * 2.220446049250313e-16 * fabs(mu), 1e-300);
    for (int r = tid; r < n; r += NTR) x[r] = 1.0 + 0.01 * (double)((r * 7 + k * 13) % 17);
    double A[Q][Q];  // LU factors of the Schur matrix (multipliers below the diagonal)
    int piv[Q];
#pragma unroll
    for (int iter = 0; iter < 2; ++iter) {
      constexpr int NS = Q * (Q + 1) / 2;
      double rp[Q], Sp[NS];  // packed lower triangle
#pragma unroll
      for (int i = 0; i < Q; ++i) rp[i] = 0.0;
#pragma unroll
      for (int e = 0; e < NS; ++e) Sp[e] = 0.0;
      for (int r = tid; r < nH; r += NTR) {
        double d = Lam[r] - sigma;
        if (d == 0.0) d = 1e-300;
        const double inv = 1.0 / d;
        const double xr = x[r];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          rp[i] += Z[r * Q + i] * xr * inv;
          if (iter == 0) {
#pragma unroll
            for (int j = 0; j <= i; ++j) Sp[tri(i, j)] += Z[r * Q + i] * Z[r * Q + j] * inv;
          }
        }
      }
      // every wave sum first, then one store per wave (a store after each sum would
      // serialise the reductions)
#pragma unroll
      for (int i = 0; i < Q; ++i) rp[i] = wave_sum(rp[i]);
      if (iter == 0) {
#pragma unroll
        for (int e = 0; e < NS; ++e) Sp[e] = wave_sum(Sp[e]);
      }
      if (lane == 0) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          park_lds[wv * NV + i] = rp[i];
          if (iter == 0) {
#pragma unroll
            for (int j = 0; j <= i; ++j) park_lds[wv * NV + Q + i * Q + j] = Sp[tri(i, j)];
          }
        }
      }
      __syncthreads();
      for (int v = tid; v < (iter == 0 ? Q + Q * Q : Q); v += NTR) vals[v] = gather<NWR>(v, park_lds, NV);
      __syncthreads();
      double sol[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) sol[i] = x[nH + i] - vals[i];
      if (iter == 0) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
          for (int j = 0; j <= i; ++j) {
            A[i][j] = sW[i * Q + j] - (i == j ? sigma : 0.0) - vals[Q + i * Q + j];
            A[j][i] = A[i][j];
          }
        lu_factor<Q>(A, piv);
      }
      lu_solve<Q>(A, piv, sol);
      for (int r = tid; r < n; r += NTR) {
        if (r < nH) {
          double d = Lam[r] - sigma;
          if (d == 0.0) d = 1e-300;
          double s = x[r];
#pragma unroll
          for (int i = 0; i < Q; ++i) s -= Z[r * Q + i] * sol[i];
          x[r] = s / d;
        } else {
#pragma unroll
          for (int i = 0; i < Q; ++i)
            if (r == nH + i) x[r] = sol[i];
        }
      }
      if (k > 0) {
        double c[Q];
        for (int kp = 0; kp < k; ++kp) {
          const double* xp = X + kp * n;
          double d = 0.0;
          for (int r = tid; r < n; r += NTR) d += x[r] * xp[r];
          c[kp] = wave_sum(d);
        }
        if (lane == 0)
          for (int kp = 0; kp < k; ++kp) park_lds[wv * NV + GS_SLOT + kp] = c[kp];
        __syncthreads();
        for (int kp = 0; kp < k; ++kp) c[kp] = gather<NWR>(GS_SLOT + kp, park_lds, NV);
        for (int r = tid; r < n; r += NTR) {
          double s = x[r];
          for (int kp = 0; kp < k; ++kp) s -= c[kp] * X[kp * n + r];
          x[r] = s;
        }
      }
      double nr = 0.0;
      for (int r = tid; r < n; r += NTR) nr += x[r] * x[r];
      park(nr, NORM_SLOT, park_lds, NV);
      __syncthreads();
      const double inv = 1.0 / sqrt(gather<NWR>(NORM_SLOT, park_lds, NV));
      for (int r = tid; r < n; r += NTR) x[r] *= inv;
    }
    __syncthreads();  // the q trailing entries, written by their own threads, are read below
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
      for (int i = 0; i < Q; ++i) s -= g[i * nH + r] * sT[i];
      P.rr_y[(int64_t)k * nH + r] = s;
    }
    __syncthreads();
  }
}

// V^T stored row-major (VT[r*nH + c] = V[c*nH + r]) for coalesced row sweeps.
__global__ __launch_bounds__(256) void k_transpose(const ProbDev* probs) {
  const ProbDev& P = probs[blockIdx.y];
  const int nH = P.nH;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)nH * nH) return;
  const int r = (int)(e / nH), c = (int)(e - (int64_t)r * nH);
  P.VT[e] = P.V[(int64_t)c * nH + r];
}

}  // namespace

hipError_t launch_rr_solve(int max_q, const ProbDev* probs, int nprob, int m, int max_nH, int dst,
                           hipStream_t s) {
  const size_t shm = rr_dyn_doubles(max_nH, max_q) * sizeof(double);
  switch (max_q) {
#define MLC_RR_CASE(QQ)                                                                       \
  case QQ:                                                                                    \
    hipLaunchKernelGGL(k_rr_solve<QQ>, dim3(nprob), dim3(rr_threads<QQ>()), shm, s, probs, m, dst); \
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

hipError_t launch_transpose_v(const ProbDev* probs, int nprob, int max_nH, hipStream_t s) {
  const int64_t n = (int64_t)max_nH * max_nH;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((n + 255) / 256), nprob), dim3(256), 0, s, probs);
  return hipGetLastError();
}
