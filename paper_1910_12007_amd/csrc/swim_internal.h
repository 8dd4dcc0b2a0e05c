// swim_internal.h -- host-side interface between the C ABI (swim_capi.hip)
// and the kernel launchers (swim_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swim_math.h"

namespace swim {

// Layout of a batch of independent systems (one hydrodynamic domain each),
// all device pointers indexed by the system id s.  System s holds nswim[s]
// filaments of npt[s] points; its filaments are [sw_off[s], sw_off[s+1]) of
// the parameter table; pt_off[s] is the start of its points in the
// large-system position buffers (unused by the persistent kernel).
struct Batch {
    int64_t n_sys;
    const int64_t* pt_off;
    const int64_t* sw_off;
    const int32_t* npt;      // points per filament
    const int32_t* nswim;    // filaments per system
    const double* params;    // [n_filaments][9]
    const void* sysc;        // SysConst<T>[n_sys]
    const void* sysc64;      // SysConst<double>[n_sys] (FP32 runs: builds the kernel tables)
    const void* tab;         // FP32 runs: TabE[n_sys][TAB_N] kernel tables
};

struct Run {
    int32_t steps;
    double dt;
    int32_t obs_every;
    int32_t n_obs;
    double eps_over_ds;
    // early rejection against a known tolerance (persistent kernel, one
    // swimmer per system): with stop_data ([n_obs][2] head data) set, a run
    // stops with SWIM_ST_REJECTED_ once the running sum of its squared head
    // deviations exceeds stop_ssq (the sum only grows, so its final
    // distance exceeds the tolerance)
    const double* stop_data = nullptr;
    double stop_ssq = 0.0;
};

// all launchers return hipError_t of the launch
// (dtype 0 also writes the FP64 constants into sysc64, for the kernel tables)
// blob: 0 the kernel reading's blob, 1 the paper's blob (closed forms at
// alpha = 0, quadrature for alpha > 0)
hipError_t launch_sysconst_batch(int dtype, int64_t n_sys, const int64_t* sw_off, const int32_t* npt,
                                 const double* params, double eps_over_ds, void* sysc, void* sysc64,
                                 int32_t* status, int blob, hipStream_t st);
hipError_t launch_sysconst(int dtype, int64_t n_sys, const double* alpha, const double* eps,
                           void* sysc, void* sysc64, int blob, hipStream_t st);
hipError_t launch_pair_velocity(int dtype, int tpl, int64_t n_blocks, const int64_t* blk_sys,
                                const int64_t* blk_first, const int64_t* pt_off, const void* sysc,
                                const void* tab, const void* x, const void* y, const void* fx,
                                const void* fy, void* ux, void* uy, hipStream_t st);
// bytes of one system's FP32 kernel table
size_t table_bytes();
// FP32 kernel tables of systems [s0, s0 + n) (FP64 constants sysc64) into tab[s]
hipError_t launch_table_build(int64_t s0, int64_t n, const void* sysc64, void* tab, int blob, hipStream_t st);
hipError_t launch_forces(int dtype, int64_t n_fil, const int64_t* fil_off, const int32_t* npt,
                         const double* params, double t, const void* x, const void* y, void* fx,
                         void* fy, hipStream_t st);
// persistent forward run, one workgroup of wps wavefronts per system
// (systems of at most 64*tpl points; tpl in {1,2,3,4,6,8}, wps in {1,2,4})
hipError_t launch_forward(int dtype, int tpl, int wps, int n_blocks, const Batch& b,
                          const Run& r, const int32_t* order, int32_t* queue, void* obs,
                          void* speed, int32_t* status, int32_t* steps_done, hipStream_t st);
// smallest waves per system of the persistent kernel for tpl targets per lane
int forward_min_wps(int tpl);
size_t forward_lds_bytes(int dtype, int tpl, int wps);
// set the kernels' dynamic-LDS limits ahead of launches (needed before a
// stream capture, in which the launch itself must not change attributes)
hipError_t prepare_forward(int dtype, int tpl, int wps);
hipError_t prepare_big_step(int dtype, int tpl, int32_t max_pts);
int forward_blocks_per_cu(int dtype, int tpl, int wps);
// one forward-Euler step of large systems, targets split over workgroups
struct BigState {
    void* xh[2];   // position hi parts, double-buffered, [n_points] T
    void* yh[2];
    void* xl[2];   // lo parts
    void* yl[2];
    void* head0;   // [n_filaments][2] T, initial head positions
};
// the symmetric FP32 large-system step: tile pairs (pairs kernel) or tiles
// (update kernel) of BIG_T = 256 points, and the partial-sum slots
struct BigTiles {
    const int64_t* sys;   // [n_items] system
    const int32_t* tile;  // [n_items] ta | tb << 16 (tile pairs, ta <= tb), or the tile
    const int64_t* poff;  // [n_sys] first partial slot of a large system (nt * nt slots)
    void* part;           // slots of 256 double pairs: slot poff + t * nt + q = tile t's sums over tile q
};
constexpr int BIG_TILE_POINTS = 256;
size_t big_pair_lds_bytes();
hipError_t prepare_big_pairs();
hipError_t launch_big_pairs(int64_t n_pairs, const BigTiles& bt, const Batch& b, const BigState& s, int step,
                            const Run& r, const int32_t* status, hipStream_t st);
hipError_t launch_big_update(int64_t n_tiles, const BigTiles& bt, const Batch& b, const BigState& s, int step,
                             const Run& r, void* obs, int32_t* status, int32_t* steps_done, hipStream_t st);
hipError_t launch_big_init(int dtype, const int64_t* list, int64_t n_list, const Batch& b,
                           const BigState& s, int32_t* status, void* obs, int32_t n_obs,
                           hipStream_t st);
hipError_t launch_big_step(int dtype, int tpl, int64_t n_blocks, const int64_t* blk_sys,
                           const int64_t* blk_first, int32_t max_pts, const Batch& b,
                           const BigState& s, int step, const Run& r, void* obs, int32_t* status,
                           int32_t* steps_done, hipStream_t st);
hipError_t launch_big_finish(int dtype, const int64_t* list, int64_t n_list, const Batch& b,
                             const BigState& s, int buf, const Run& r, void* speed,
                             const int32_t* status, int32_t* steps_done, hipStream_t st);
size_t big_step_lds_bytes(int dtype, int32_t max_pts);

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
hipError_t launch_abc_distance(int dtype, int64_t n, int32_t n_obs, const void* obs,
                               const double* data, const int32_t* status, double* dist,
                               hipStream_t st);
// k-th smallest (1-based) of n doubles -> *out (device); single workgroup radix select
hipError_t launch_select_kth(int64_t n, const double* v, double q, double* out, hipStream_t st);
hipError_t launch_accept(int64_t n, const double* dist, const double* tol, uint8_t* acc,
                         hipStream_t st);
hipError_t launch_gauss_loglik(int dtype, int64_t n, int32_t n_obs, const void* obs, const double* data,
                               const double* sigma, const int32_t* status, double* logl, hipStream_t st);

// surrogate MLP (swim_mlp.hip)
// operands of the GEMM epilogues (unused ones may be null)
struct GemmEpi {
    const float* bias = nullptr;  // [N]
    float* aux = nullptr;         // GELU: H out; DGELU: pre-activations in; MSE: dY out
    const float* T = nullptr;     // MSE: targets [M][N]
    float* sq = nullptr;          // MSE: squared errors out [M][N]
    float sc = 0.0f;              // MSE: 2 / (M N)
};
// workspace of the split-K partial sums
struct MlpWs {
    float* part = nullptr;
    int64_t part_floats = 0;
};
// epi: 0 plain, 1 bias + GELU, 2 bias, 3 times GELU', 4 bias + MSE gradient
hipError_t launch_gemm_bf16(int epi, int M, int N, int K, const float* A, int64_t sam, int64_t sak,
                            const float* B, int64_t sbk, int64_t sbn, float* C, int64_t ldc,
                            const GemmEpi& E, const MlpWs& ws, hipStream_t st);
hipError_t launch_colsum(int M, int N, const float* A, int64_t lda, float* out, hipStream_t st);
hipError_t launch_sum(int64_t n, const float* v, float* out, hipStream_t st);
hipError_t launch_gather_rows(int M, const int32_t* perm, int64_t nrows, const float* X, int nx,
                              const float* T, int nt, float* Xb, float* Tb, hipStream_t st);
hipError_t launch_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1,
                       float b2, float c1, float c2, float eps, hipStream_t st);
hipError_t launch_prescreen(int M, int N, int n_sum, const float* Y, const float* mu,
                            const float* sd, const float* obs, float tol, float* dist,
                            uint8_t* keep, hipStream_t st);
hipError_t launch_compact(int64_t n, const uint8_t* keep, int32_t* counts, int64_t* idx,
                          int64_t* total, hipStream_t st);
hipError_t launch_features(int64_t n, const double* theta, double b, double om, const float* mu,
                           const float* sd, float* X, hipStream_t st);
hipError_t launch_targets(int dtype, int64_t n, int n_obs, const void* obs, const void* speed,
                          double x0, double y0, const int32_t* idx, int n_sum, float* T,
                          hipStream_t st);
hipError_t launch_colstats(int64_t n, int cols, const float* A, float* mu, float* sd, hipStream_t st);
hipError_t launch_standardize(int64_t n, int cols, float* A, const float* mu, const float* sd,
                              hipStream_t st);
hipError_t launch_prior_draw(uint64_t seed, int64_t n, const double* lo, const double* hi,
                             double* theta, hipStream_t st);
hipError_t launch_param_rows(int64_t cap, const int64_t* n_dev, const int64_t* idx, int64_t n_theta,
                             const double* theta, double b, double om, double kw, double* rows,
                             hipStream_t st);
hipError_t launch_gather_f32(int64_t cap, const int64_t* n_dev, const int64_t* idx, int64_t n_src,
                             const float* src, int cols, float* dst, hipStream_t st);
hipError_t launch_flag_eq(int64_t n, const int32_t* v, int32_t want, uint8_t* keep, hipStream_t st);
hipError_t launch_flag_bounded(int64_t n, const float* T, int nt, int n_disp, float max_disp, uint8_t* keep,
                               hipStream_t st);

// fused MLP inference (mode 0: outputs Y[M][33]; mode 1: prescreen distance
// and keep flag), from the bfloat16 weight copy W16 (launch_pack_w16)
size_t mlp_fused_lds_bytes();
int64_t mlp_w16_count();
hipError_t launch_pack_w16(const float* P, uint16_t* W16, hipStream_t st);
hipError_t launch_mlp_fused(int mode, int64_t M, const float* X, const uint16_t* W16, const float* P, float* Y,
                            const float* out_mu, const float* out_sd, const float* obs, int n_sum, float tol,
                            float* dist, uint8_t* keep, hipStream_t st);

// full sperm model (swim_sperm.hip): shape shared by all systems of a call
struct SpermShape {
    int32_t nf, nh, nsw, pad;   // flagellum points, head points, swimmers per system
    double ds, ch, hr, dn, dth; // 1/(nf-1), head chord, head radius, neck gap, 2 pi/nh
    double eps;                 // blob width
    double L0[5];               // neck rest lengths (last flagellum point to pi-dth, pi,
                                // pi+dth; the one before to pi-dth, pi+dth)
};
struct SpermRun {
    int64_t n_sys;
    const double* sysp;  // [n_sys][SWIM_SP_NPARAM]
    const double* swp;   // [n_sys * nsw][3]: x0, y0, phase
    int32_t steps, obs_every, n_obs, pad;
    double dt;
};
hipError_t launch_sperm_setup(int dtype, int64_t n_sys, int32_t nsw, double eps, const double* sysp,
                              const double* swp, void* sysc, void* sysc64, int32_t* status, int blob,
                              hipStream_t st);
size_t sperm_lds_bytes(int dtype, int tpl, int wps);
hipError_t prepare_sperm(int dtype, int tpl, int wps);
int sperm_blocks_per_cu(int dtype, int tpl, int wps);
// persistent run, one workgroup of wps wavefronts per system (tpl in
// {1,2,3,4,6,8}, wps in {2,4,8})
hipError_t launch_sperm_forward(int dtype, int tpl, int wps, int nblocks, const SpermShape& g, const SpermRun& r,
                                const void* sysc, const void* tabs, int32_t* queue, void* head, void* tail,
                                int32_t* status, hipStream_t st);
// observables per system and sample k = 1..n_obs into g[n_sys][n_obs][2]:
// kind 0 head-centre velocity of swimmer 0, kind 1 (tail, head) distances of
// swimmers 0 and 1
hipError_t launch_sperm_observables(int dtype, int kind, int64_t n_sys, int32_t nsw, int32_t n_obs, double dt_obs,
                                    const void* head, const void* tail, const int32_t* status, double* g,
                                    hipStream_t st);
// Gaussian log-likelihood with standard deviations sig2[i][0] (entries 0,
// 2, ...) and sig2[i][1] (entries 1, 3, ...); status may be NULL
hipError_t launch_gauss_loglik2(int64_t n, int32_t n_obs, const double* g, const double* data, const double* sig2,
                                const int32_t* status, double* logl, hipStream_t st);

// velocity and pressure at arbitrary points (swim_field.hip): constants of one
// fluid and blob.  The pressure weight m(r) / (2 pi r^2) is inv_2pi / R^2
// (stokes), the power series ser[] in delta = r^2/eps^2 for delta < 1/4, and
// inv_2pi (1 - eps K1(alpha R) / (R K1e)) / r^2 otherwise.
constexpr int FIELD_NSER = 26;
struct FieldConst {
    SysConst<float> c32;
    SysConst<double> c64;
    double h1c, inv_e2, e2, eps, alpha, K1e, inv_2pi;
    int32_t stokes, paper;  // paper: the paper's blob (mass 1 - eps^3/R^3)
    double ser[FIELD_NSER];
};
hipError_t launch_flow_field(int dtype, int64_t n, const void* x, const void* y, const void* fx, const void* fy,
                             const FieldConst& fc, int64_t nt, const void* tx, const void* ty, void* u, void* v,
                             void* p, const void* tab, void* wtab, hipStream_t st);

}  // namespace swim
