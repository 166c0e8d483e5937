// Kernel launchers of libmlc (host side).  Every launcher enqueues on the given stream
// and returns the launch status.  Grids span the largest problem of a batch; blocks of
// problems that are smaller, or that have no level m, exit at once.
#pragma once
#include <hip/hip_runtime.h>
#include "mlc_device.h"

// ---- one correction step (Algorithm 4.1) at level m, ping-pong src -> dst ----
hipError_t launch_prolong_residual(int kind, const ProbDev* probs, int nprob, int m, int src,
                                   int64_t max_nodes, int max_q, hipStream_t s);
hipError_t launch_local_pcg(int kind, int nt, const ProbDev* probs, const TileItem* items,
                            int nitems, char* store, const double* inv, int m, ItemStat* stats,
                            double rtol, int max_it, int nu, double omega, double omega2,
                            int64_t rhs_in_tile,
                            int max_tile_nx, hipStream_t s);
hipError_t launch_local_mixed(int kind, int nt, const ProbDev* probs, const TileItem* items,
                              int nitems, char* store, const double* inv, int m, ItemStat* stats,
                              double rtol, int max_it, int max_refine, double inner_rtol, int nu,
                              double omega, double omega2, int max_tile_nx, hipStream_t s);
// Algorithm 4.1 step 2 as stated (MLC_POU_INTERFACE), single problem: u~ from the tile
// solutions on the closed G_j and a global CG on the rest, preconditioned by a multigrid
// V-cycle on that region (vec: skel_stride(nc, L) doubles per right-hand side, parts: 2 per
// 16 x 16 nodes (rounded up per side) of level m per right-hand side, scal: 8 doubles per right-hand side, rec: 2
// doubles that receive the maximum over right-hand sides of the iterations and of the final
// ||r|| / ||r_0||).  poll: stop when every right-hand side has converged (the stream is
// synchronised every 4 iterations to read the flags) or after max_it iterations; otherwise
// enqueue exactly max_it iterations (converged right-hand sides frozen), with no host
// synchronisation, e.g. for graph capture.
hipError_t run_interface_gluing(int kind, const ProbDev* dprob, const TileItem* items,
                                const int32_t* sub_item, const char* store, int m, int q, int nc,
                                int64_t stride, double rtol, int max_it, bool poll, double* vec,
                                double* parts, double* scal, double* rec, hipStream_t s);
int64_t skel_stride(int nc, int L);

// Widest tile row (interior nodes) whose banded smoothing passes fit the device's
// per-workgroup LDS with nt threads (three rings of nt/64 + 2 rows, plus the LDS tail of
// the V-cycle when with_tail), capped at the widest tile of the launch; 0 when nu != 2 or
// nothing fits.  *cap2 receives the same for bands of two rows per wave (rings of
// 2 nt/64 + 2 rows), *lds the bytes to allocate.
int ring_capacity(int nt, int nu, int max_tile_nx, int elem_bytes, bool with_tail, size_t* lds,
                  int* cap2);
// The rings of a launch: ring_capacity with the LDS V-cycle tail for 1024 threads, and in
// *cap2n the widest tile that takes two band rows per wave when it gives the tail up (0
// when that adds nothing); *lds covers both layouts.  Every cap depends on the device only
// (or is at least the widest tile), so each item's choice depends on its own width alone.
int ring_layout(int nt, int nu, int max_tile_nx, int elem_bytes, size_t* lds, int* cap2,
                int* cap2n);
// Elements of the ring region for nw waves and the two caps above (the tail follows it).
__host__ __device__ inline long ring_elems(int nw, int cap1, int cap2) {
  const long a = 3L * (nw + 2) * cap1, b = 3L * (2 * nw + 2) * cap2;
  return a > b ? a : b;
}
hipError_t launch_pou_glue(const ProbDev* probs, int nprob, const TileItem* items,
                           const int32_t* sub_item, const char* store, int m, int64_t max_nodes,
                           int max_q, hipStream_t s);
hipError_t launch_rr_apply(int kind, const ProbDev* probs, int nprob, int m, int64_t max_nodes,
                           int max_q, hipStream_t s);
hipError_t launch_restrict(const ProbDev* probs, int nprob, int l, int m, int64_t max_nodes_l,
                           int max_q, hipStream_t s);
hipError_t launch_rr_project(const ProbDev* probs, int nprob, int max_nH, int max_q,
                             hipStream_t s);
hipError_t launch_rr_solve(int max_q, const ProbDev* probs, int nprob, int m, int max_nH, int dst,
                           hipStream_t s);
hipError_t launch_transpose_v(const ProbDev* probs, int nprob, int max_nH, hipStream_t s);
hipError_t launch_rr_combine(const ProbDev* probs, int nprob, int max_nc1sq, int max_q,
                             hipStream_t s);
hipError_t launch_assemble(const ProbDev* probs, int nprob, int m, int dst, int64_t max_nodes,
                           int max_q, hipStream_t s);

// ---- setup ----
hipError_t launch_coarsen_kappa(const double* lo_f, const double* up_f, double* lo_c,
                                double* up_c, int Nc, hipStream_t s);
// Coefficient kind 3: seven-point stiffness and mass planes of the finest level from the
// per-triangle tensor and weight, and of a coarser level by the Galerkin product.
hipError_t launch_tensor_fine(const double* coef, double* st, float* stf, int N, double h2,
                              hipStream_t s);
hipError_t launch_galerkin7(const double* fine, double* coarse, float* coarsef, int Nc,
                            hipStream_t s);
hipError_t launch_coarse_matrices(int kind, const ProbDev* probs, int nprob, int max_nH,
                                  hipStream_t s);
// Full generalized eigendecomposition of the coarse matrices of every problem whose eig_ws
// is set (Cholesky, two-sided Jacobi, back substitution; one workgroup per problem).
hipError_t launch_coarse_eig(const ProbDev* probs, int nprob, hipStream_t s);
hipError_t launch_init_u0(const ProbDev* probs, int nprob, int dst, int max_nc1sq, hipStream_t s);
hipError_t launch_tile_inverse(int kind, const ProbDev* probs, const TileItem* items,
                               int nitems, double* inv, hipStream_t s);

// ---- state in/out ----
hipError_t launch_output_signed(const double* u, int64_t nn, int q, double* parts, double* out,
                                hipStream_t s);
hipError_t launch_set_state(const ProbDev* prob, int level, int dst, const double* in,
                            int64_t nn, hipStream_t s);

// ---- adjoint (reverse sweep) ----
hipError_t launch_tape_tiles(const TileItem* items, int nitems, const char* store, int m, double* te,
                             const int64_t* te_off, hipStream_t s);
hipError_t launch_restrict1(const ProbDev* p, const double* in, double* out, int l, int64_t nodes_l,
                            hipStream_t s);
hipError_t launch_coarse_project(const ProbDev* p, int nH, const double* a, double* out,
                                 hipStream_t s);
hipError_t launch_coarse_combine(const ProbDev* p, int nc1sq, const double* y, double* grid,
                                 hipStream_t s);
hipError_t launch_dot_sum(const ProbDev* p, int m, int64_t nodes, const double* a, const double* b,
                          bool mass, double* parts, double* out, hipStream_t s);
hipError_t launch_adj_rr(const ProbDev* p, const double* rr, const double* cbar_H,
                         const double* cbar_u, const double* lam_bar, double* y, double* coef,
                         hipStream_t s);
hipError_t launch_adj_shat(const ProbDev* p, int m, int64_t nodes, const double* ygrid,
                           const double* coef, const double* ut, double* shat, hipStream_t s);
hipError_t launch_adj_utbar(int kind, const ProbDev* p, int m, int64_t nodes, const double* u,
                            const double* shat, const double* ubar_m, const double* coef,
                            const double* rr, double* out, hipStream_t s);
hipError_t launch_adj_tile_rhs(const ProbDev* p, const TileItem* items, int nitems,
                               const int32_t* sub_item, char* store, int m, const double* utbar,
                               hipStream_t s);
hipError_t launch_adj_rbar(const ProbDev* p, const TileItem* items, const int32_t* sub_item,
                           const char* store, int m, int64_t nodes, double* rbar, hipStream_t s);
hipError_t launch_adj_next(int kind, const ProbDev* p, int m, int64_t nodes, const double* uk,
                           const double* lam_k, const double* utbar, const double* rbar,
                           double* ubar, double* next, hipStream_t s);
hipError_t launch_adj_products(const ProbDev* p, int m, int64_t cells, const double* u,
                               const double* c_uu, const double* shat, const double* rbar,
                               const double* ubar, const TileItem* items, const int32_t* sub_item,
                               const char* store, const double* te, const int64_t* te_off,
                               double* klo, double* kup, hipStream_t s);
hipError_t launch_adj_level0(const ProbDev* p, int nH, const double* ubar0, double* a,
                             hipStream_t s);
hipError_t launch_adj_down(const double* plo, const double* pup, double* clo, double* cup, int Nc,
                           hipStream_t s);
hipError_t launch_adj_out(const double* lo, const double* up, int N, int kind, int nc, double* out,
                          hipStream_t s);
