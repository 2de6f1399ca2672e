// amc_kernels.hpp -- host-callable launchers of the device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "amc_dev.hpp"

namespace amc {

// One wavefront per (r, s): LDS mode (realized graph in LDS) and L2 mode
// (realized graph, B and labels in a per-workgroup global scratch); dist16
// selects 16-bit distance entries in the wavefront regions.
uint32_t lds_bytes_wave(int n, uint32_t adj_cap, uint32_t adj_bytes, int waves, bool dist16, uint32_t *wave_bytes);
// sg: L2 mode with each wavefront's path counts in the workgroup's global
// scratch (lane-per-vertex mappings 1 / 2 / 3 only); l2_scratch_words then
// counts sg_waves such arrays.
uint32_t lds_bytes_wave_l2(int n, int waves, bool dist16, bool b_global, bool sg, uint32_t *wave_bytes);
size_t l2_scratch_words(int n, uint32_t adj_cap, uint32_t adj_bytes, int sg_waves);
hipError_t launch_sweep_wave(const LaunchCtl &LC, bool weighted, bool l2, bool dist16, bool sg, int group,
                             uint32_t adj_bytes, int blocks, int waves, uint32_t lds, hipStream_t st);

// Workgroup-per-(r, s) sweep with frontier queues (graphs beyond the LDS mode).
uint32_t lds_bytes_block(int n, int threads);
uint32_t block_staging_bytes(int n);
// state_place: where the per-source state (distances, path counts, order,
// B, labels, row offsets) lives: 0 LDS, 1 the workgroup's scratch except the
// distances and row offsets (lds_bytes_block_hybrid bytes of LDS), 2 all in
// the workgroup's scratch
uint32_t lds_bytes_block_hybrid(int n);
size_t block_scratch_words(int n, int64_t m, bool weighted, int state_place = 0);
hipError_t launch_sweep_block(const LaunchCtl &LC, bool weighted, int state_place, int blocks, int threads,
                              uint32_t lds, hipStream_t st);

hipError_t set_sweep_wave_attrs(int max_lds);
hipError_t set_sweep_block_attrs(int max_lds);

// Robust tail (sampled admissible kernels, sensitivity, transition rewards).
hipError_t robust_perturb(int n, const double *Q0, uint64_t seed, int sample, const int *sample_ptr, double delta,
                          double r_min, double *Q, double *A, hipStream_t st);
hipError_t robust_perturb_batch(int n, const double *Q0, uint64_t seed, int sample0, int batch, double delta,
                                double r_min, double *A, size_t stride, hipStream_t st);
hipError_t robust_divergence(int n, int batch, const double *b, const double *b0, double *kl, double *tv,
                             hipStream_t st);
hipError_t robust_normalize_rows(int n, int batch, const double *mu, double *b, hipStream_t st);
hipError_t robust_argmax(int m, const double *x, int *out, hipStream_t st);
hipError_t robust_gather_row(int n, const double *rows, const int *idx, double *dst, hipStream_t st);
hipError_t robust_vecmat(int n, const double *x, const double *M, double *y, hipStream_t st);
hipError_t robust_blin(int n, const double *b0, const double *mu0, const double *v, double *b_lin, hipStream_t st);
hipError_t robust_axpy(size_t count, const double *A, double alpha, const double *B, double beta, const double *D,
                       double *C, hipStream_t st);
hipError_t robust_infnorm(int n, const double *A, unsigned long long *out, hipStream_t st);
hipError_t robust_gemm(int n, const double *A, const double *B, double *C, hipStream_t st);
hipError_t robust_rem_bound(const unsigned long long *norms, double *out, hipStream_t st);
hipError_t robust_trans_rewards(int n, const double *Q, const double *f, double *psw, double *pimp, hipStream_t st);
size_t w1_lds_bytes(int n);
hipError_t robust_w1(int n, int m, const int32_t *eu, const int32_t *ev, const uint32_t *len, const int32_t *rp,
                     const int32_t *inc, int batch, const double *P, const double *q, double *fscr, double *w1, int *err,
                     hipStream_t st);

// Anchored r-hop neighbourhoods (LDS mode only).
uint32_t lds_bytes_anchored(int n, uint32_t adj_cap, uint32_t adj_bytes, int waves, uint32_t *wave_bytes);
hipError_t set_anchored_attrs(int max_lds);
hipError_t launch_anchored(const LaunchCtl &LC, bool weighted, uint32_t adj_bytes, int blocks, int waves, uint32_t lds,
                           hipStream_t st);

// Trajectory simulator (LDS mode only).
hipError_t set_traj_attrs(int max_lds);
// L2 placements of the trajectory kernel (realized graph in a per-workgroup
// global scratch): LDS bytes before the wavefront regions, i.e. B(H) f64[n]
// unless b_global, and the component list u16[n].  place: 0 = LDS layout,
// 1 = L2 with B in LDS, 2 = L2 with B in the scratch.
uint32_t traj_l2_lds_base(int n, bool b_global);
hipError_t launch_traj(const TrajArgs &T, bool weighted, bool dist16, int place, int group, uint32_t adj_bytes, int blocks,
                       int waves, uint32_t lds, hipStream_t st);
hipError_t traj_estimates(int n, int episodes, int max_steps, const int32_t *lengths,
                          const unsigned long long *visits, const unsigned long long *ctr, uint32_t *hist,
                          double *b_hat, double *survival, hipStream_t st);

// Finite-k Top-k stage and its tail pieces.
hipError_t set_topk_attrs(int max_lds);
uint32_t topk_lds(int n);
// bytes per workgroup of the Top-k arrays in global memory (when topk_lds(n)
// exceeds the LDS; TopkArgs.gscr set)
uint64_t topk_global_bytes(int n);
hipError_t launch_topk_reduce(const TopkArgs &A, int blocks, hipStream_t st);
hipError_t tail_div(int n, const double *x, double d, double *y, hipStream_t st);
hipError_t tail_reward_afc(int n, const double *mu, const double *scal, const double *psi, double *out,
                           hipStream_t st);
hipError_t tail_fb_counts(int n, const uint32_t *counts, const uint32_t *counts_w, int fb, uint32_t *cf,
                          hipStream_t st);
hipError_t tail_censor(int n, const double *b, const uint8_t *fb_mask, double *b_cens, double *c_out,
                       hipStream_t st);

// Tail.
hipError_t fill_u32(void *p, size_t count, uint32_t v, hipStream_t st);
hipError_t tail_kernel_from_counts(int n, const uint32_t *counts, uint32_t R, double eta, double *Q, double *r,
                                   double *A, hipStream_t st);
hipError_t tail_kernel_from_Q(int n, const double *Q, double *r, double *A, hipStream_t st);
hipError_t tail_invert(int n, double *A, int *err, hipStream_t st);
hipError_t tail_invert_batched(int n, double *A, size_t stride, int batch, int *err, hipStream_t st);
hipError_t tail_visits_batched(int n, const double *N, size_t stride, int batch, const double *s, double *mu,
                               hipStream_t st);
hipError_t tail_visits(int n, const double *N, const double *s, double *mu, double *b, const double *f,
                       const uint8_t *pool, double *b_bar, const double *r, double r_lower, int topk, int32_t *top,
                       double *scal, hipStream_t st);
hipError_t tail_certificates(int n, int topk, const double *Q, const double *N, const double *mu,
                             const int32_t *top, int32_t *cv, double eps, double r_lower, double *gap,
                             double *sharp, double *sharp_supp, uint8_t *ok, int *support, hipStream_t st);
hipError_t tail_xi(int n, const uint32_t *counts_w, uint32_t R, double *xi, hipStream_t st);

// Bootstrap of b (Section 8.4).
hipError_t boot_transpose(int n, uint32_t R, const int32_t *nt, uint16_t *tr, hipStream_t st);
hipError_t boot_rows(int n, uint32_t R, const uint16_t *tr, uint64_t seed, uint32_t beta0, int batch, bool ident,
                     double eta, double *A, size_t stride, hipStream_t st);
size_t boot_stats_lds(int B);
hipError_t boot_stats(int n, int B, const double *b_rep, int klo, int khi, double *mean, double *sd, double *lo,
                      double *hi, hipStream_t st);

}  // namespace amc
