// Host-side launchers of the gfx950 kernels (one per kernel family).
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mrcm {

// Local problems (local_kernels.hip)
hipError_t launch_reset_status(DevStatus *st, hipStream_t s);
hipError_t launch_check_perm(const double *kx, const double *ky, const double *kz, long long n,
                             DevStatus *st, hipStream_t s);
hipError_t launch_coef(const Geom &g, int n_sub, int max_cells, double *coef, double *r0,
                       double *scal, hipStream_t s);
// queue non-null: the persistent form over a device work queue (eight
// counters, zeroed by the launcher on the stream); else one workgroup per item
hipError_t launch_factor(int fp32, const SubDesc *subs, const int *order, int n_sub,
                         const double *coef, const double *scal, void *L, void *Dg, DevStatus *st,
                         int bmax, hipStream_t s, int *queue = nullptr);
// coef non-null with a correction mode: each workgroup forms its item's
// residual into B before solving, from the right-hand sides in rhs0 (or in B
// itself when rhs0 is null, which then serves a single sweep)
hipError_t launch_solve(int fp32, const Geom &g, const int4 *work, int n_work, const double *scal,
                        const void *L, const void *Dg, double *B, double *X, int mode, int bmax,
                        hipStream_t s, const double *coef = nullptr, const double *rhs0 = nullptr,
                        int *queue = nullptr);
// B2: a second copy of the right-hand sides, or null
// mmax: the largest column count m over the subdomains
hipError_t launch_rhs(const Geom &g, int n_sub, int max_cells, int mmax, const double *r0, double *B,
                      hipStream_t s, double *B2 = nullptr);
int solve_chunk_max();
size_t factor_lds_bytes(int fp32, int bmax);
size_t solve_lds_bytes(int fp32, int bmax, int mmax);
// subs: the subdomains to take (n_sub of them), or null for 0 .. n_sub-1
hipError_t launch_residual(const Geom &g, int n_sub, int max_cells, int mmax, const double *coef,
                           const double *r0, const double *X, double *R, double *norms,
                           hipStream_t s, const int *subs = nullptr);
int solve_blocks_per_cu(int fp32, int bmax);
int factor64_blocks_per_cu(int bmax);
int factor32_blocks_per_cu(int bmax);
hipError_t launch_ir_check(const double *norms, int ncols, double *out, hipStream_t s);
hipError_t launch_flux(const Geom &g, int n_sub, const double *X, double *F, double *Fb,
                       double *SAb, hipStream_t s);

// Reconstruction by re-solve: one right-hand side per subdomain (B, X, R at
// each subdomain's cell offset), its residual from the coefficients, and the
// scatter of the solution into the global pressure.
hipError_t launch_resolve_rhs(const Geom &g, int n_sub, int max_cells, const double *r0, const double *pi, int nv,
                              double *B, hipStream_t s);
hipError_t launch_resolve_residual(const Geom &g, int n_sub, int max_cells, const double *coef, const double *B,
                                   const double *X, double *R, hipStream_t s);
hipError_t launch_resolve_scatter(const Geom &g, int n_sub, int max_cells, const double *X, double *p,
                                  hipStream_t s);

// Mean post-processing: the per-subdomain Neumann coefficients and
// right-hand side (B, and a copy in X for the in-place solve) from the
// multiscale velocity U, and the post-processed pressure and velocity.
hipError_t launch_mean_coef(const Geom &g, int n_sub, int max_cells, const double *U, double *coef, double *B,
                            double *X, double *scal, hipStream_t s);
hipError_t launch_mean_velocity(const Geom &g, const double *U, const double *P, double *pt, double *Ut,
                                hipStream_t s);

// Saturation step of the two-phase run (transport_kernels.hip): the step,
// its CFL time step into a device scalar, and K lambda(S).
hipError_t launch_transport(const TwoPhaseGrid &t, const double *U, const double *q, const double *S,
                            const double *dt, double *Sout, hipStream_t s);
// The fused step in three launches: clear dt_next's accumulator, the step
// with the CFL speed of its result, turn the accumulator into the step.
hipError_t launch_speed_clear(double *dt, hipStream_t s);
hipError_t launch_transport_fused(const TwoPhaseGrid &t, const double *U, const double *q, const double *S,
                                  const double *dt, double *Sout, double *dt_next, hipStream_t s,
                                  const unsigned char *src_tiles = nullptr);
hipError_t launch_speed_finish(const TwoPhaseGrid &t, double cfl, double dt_max, double *dt, hipStream_t s);
// Tiles of the saturation step, and their marks where q has a source (for
// launch_transport_fused's src_tiles: q is then read in those tiles only).
long long transport_tile_count(const TwoPhaseGrid &t);
hipError_t launch_source_tiles(const TwoPhaseGrid &t, const double *q, unsigned char *flags, hipStream_t s);
hipError_t launch_transport_dt(const TwoPhaseGrid &t, const double *U, const double *S, double cfl, double dt_max,
                               double *dt, hipStream_t s);
hipError_t launch_mobility(const TwoPhaseGrid &t, const double *S, const double *kx, const double *ky,
                           const double *kz, double *ox, double *oy, double *oz, hipStream_t s);

// Conjugate-gradient form of the local solves (pcg_kernels.hip).  One
// workgroup per column (subdomain by col_sub); X0 null for a zero start.
int pcg_max_cells();
hipError_t launch_pcg(const Geom &g, const int *col_sub, int ncols, int max_cells, const double *coef,
                      const double *scal, const double *B, const double *X0, double *X, int max_iter, double tol,
                      int x0_scale, int *iters, int *conv, hipStream_t s);

// Network of the learned warm start (nn_kernels.hip)
int conv3d_max_channels();
hipError_t launch_conv3d(const float *x, const float *w, const float *bias, float *y, const float *mask, int B,
                         int Cin, int Cout, int D, int H, int W, int dil, int relu, hipStream_t s);
hipError_t launch_conv3d_flip(const float *w, float *wt, int Cin, int Cout, hipStream_t s);
hipError_t launch_conv3d_wgrad(const float *x, const float *dy, float *dw, float *db, int B, int Cin, int Cout,
                               int D, int H, int W, int dil, hipStream_t s);
// Most partial sums of the loss (one per workgroup of 256 threads).
constexpr int kMsePartialsMax = 1024;
// Devices for which the allocation-free entry point keeps a scratch address.
constexpr int kMaxDevices = 64;
int mse_partials(long long n);
// As launch_mse, with the partial sums in the library's static per-device
// array instead of a caller's workspace: allocates nothing.
hipError_t launch_mse_static(const float *y, const float *t, float *dy, double *loss, long long n,
                             hipStream_t s);
hipError_t launch_mse(const float *y, const float *t, float *dy, double *part, double *loss, long long n,
                      hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, int t, float lr, float b1, float b2,
                       float eps, hipStream_t s);
hipError_t launch_nn_features(const Geom &g, const int *sel, const int *sample0, int n_sel, int mmax,
                              const double *R, const double *X, int V, float *inp, float *tgt, hipStream_t s);
hipError_t launch_nn_scatter(const Geom &g, const int *sel, const int *sample0, int n_sel, int mmax,
                             const float *out, int V, double *x0, hipStream_t s);

// Encoder-decoder network of the learned warm start (unet_kernels.hip);
// activations FP32 channels last, convolutions on BF16 MFMA.
int unet_pad16(int c);
int unet_max_channels();
hipError_t launch_unet_pack(const float *w, unsigned short *wf, unsigned short *wt, int cin, int cout, hipStream_t s);
hipError_t launch_unet_conv(const float *x, const unsigned short *wf, const float *bias, float *y, const float *mask,
                            int batch, int d, int h, int w, int cin, int cout, int relu, hipStream_t s);
long long unet_wgrad_workspace(long long nvox, int cin, int cout);
hipError_t launch_unet_wgrad(const float *x, const float *dy, float *dw, float *db, float *work, int batch, int d,
                             int h, int w, int cin, int cout, hipStream_t s);
hipError_t launch_unet_pool(const float *x, float *y, int batch, int d, int h, int w, int c, int backward,
                            hipStream_t s);
hipError_t launch_unet_up(const float *x, float *y, int batch, int d, int h, int w, int c, int backward,
                          hipStream_t s);
hipError_t launch_unet_relu_mask(float *g, const float *out, long long n, hipStream_t s);
hipError_t launch_channels_last(const float *in, float *out, int batch, int c, long long v, hipStream_t s);

// Interface system and reconstruction (iface_kernels.hip)
hipError_t launch_fill(double *a, long long n, double v, hipStream_t s);
hipError_t launch_copy(const double *a, double *b, long long n, hipStream_t s);
hipError_t launch_iface_scatter(const Geom &g, int n_sub, const int *patches, const int *pos,
                                const double *F, const double *Fb, const double *SAb, double *AB,
                                int w, double *b, hipStream_t s);
size_t ldl_inv_size(int n);
hipError_t launch_band_ldl(const double *AB0, double *AB, const double *b0, double *b, double *y, int n, int w,
                           double *inv, DevStatus *st, hipStream_t s);
hipError_t launch_lu_sweep(const double *AB, const double *inv, int n, int w, double *x, int upper,
                           hipStream_t s);
hipError_t launch_band_residual(const double *AB, int n, int w, const double *x, const double *b,
                                double *r, int flip, hipStream_t s);
hipError_t launch_perm(const double *src, const int *pos, int nv, double *dst, int to_natural,
                       hipStream_t s);
hipError_t launch_norm2(const double *v, int n, double *out, hipStream_t s);
hipError_t launch_axpy(double *y, const double *x, int n, hipStream_t s);
hipError_t launch_recon_p(const Geom &g, int n_sub, const int *patches, const double *X,
                          const double *pi, int nv, double *p, hipStream_t s);
hipError_t launch_recon_u(const Geom &g, const double *p, const double *pi, int nv, double *U,
                          hipStream_t s);

}  // namespace mrcm
