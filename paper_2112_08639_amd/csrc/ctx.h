// The libdk context and the internal entry points shared by the HIP sources.
#pragma once

#include <string>
#include <vector>

#include "../../include/dk.h"
#include "common.h"

struct dk_ctx {
  // grid
  int nx = 0, ny = 0, nz = 0;
  long ngrid = 0;
  double lx = 0, ly = 0, lz = 0, hx = 0, hy = 0, hz = 0, dv = 0;  // dv = hx*hy*hz
  int precision = DK_PREC_FP64;
  int device = 0;
  hipStream_t stream = nullptr;

  // local potential
  double* veff64 = nullptr;
  float* veff32 = nullptr;
  double vmax = 0.0;
  bool have_potential = false;

  // projectors: dense column-major N_grid x n_proj tables (ld = ngrid)
  int n_proj = 0, n_atoms = 0;
  double* chi64 = nullptr;
  float* chi32 = nullptr;
  // mixed path, dense integrals over more than 64 projectors: the three bf16
  // pieces of the table (split_planes layout, k = grid point), built with it
  void* chi_pieces = nullptr;
  size_t chi_pieces_bytes = 0;
  double* dchi64 = nullptr;  // grad_h chi along x, y, z: 3 tables following chi64 in one allocation
  float* dchi32 = nullptr;
  double* gamma_dev = nullptr;
  int* atom_dev = nullptr;
  std::vector<double> gamma_h;
  std::vector<int> atom_h;
  double nl_bound = 0.0;  // sum over gamma_p > 0 of gamma_p h^3 |chi_p|^2
  // block mask of the tables: mask_t[pt*mask_t_stride + gb] for 64-projector
  // tiles x 64-point grid blocks
  uint8_t* mask_t = nullptr;
  long mask_t_stride = 0;
  // per 64-point grid block, the 4-projector groups with a nonzero table entry
  // there: klist[gb * n_groups + i] for i < kcount[gb], increasing
  int* klist = nullptr;
  int* kcount = nullptr;
  int n_groups = 0;
  // projector integrals over compact supports (gather.hip): chunks of
  // consecutive 64-point blocks {first block, blocks, union offset, union
  // length}, per (chunk, block) row the union slot -> table entry map and the
  // live 16-row blocks, the occurrences of every group among the unions, and
  // the compact (pre-split) table entries
  int n_gchunks = 0;
  long g_rows = 0;     // sum of the union lengths
  long g_entries = 0;  // (block, live group) pairs
  void* gchunk = nullptr;
  int* gqoff = nullptr;
  int* gamap = nullptr;
  unsigned* gbmask = nullptr;
  int* gocc_off = nullptr;
  int* gocc = nullptr;
  void* gtab = nullptr;
  // device-built tables (dk_set_projector_model): atom positions (3 n_atoms)
  // followed by the projector norms |chi_p|^2 (n_proj)
  double* proj_aux = nullptr;
  size_t proj_aux_len = 0;
  // the model behind device-built tables (0 channels: tables came from the
  // host, dk_set_projectors)
  int model_channels = 0;
  int model_l[DK_PROJ_MAX_CHANNELS] = {};
  double model_rc[DK_PROJ_MAX_CHANNELS] = {};
  double model_cutoff_rel = 0.0;

  // atoms of the self-consistent workloads: pseudocharge / core model, the
  // per-atom periodic factor tables and the fields b, v_core on the grid
  int n_local_atoms = 0;
  double loc_z = 0, loc_rc = 0, loc_core_amp = 0, loc_core_w2 = 0;
  double* pos_dev = nullptr;
  double* atom_tab = nullptr;
  double* b_dev = nullptr;
  double* vcore_dev = nullptr;

  // workspace (caller owned)
  char* ws = nullptr;
  size_t ws_bytes = 0;

  // per-kernel timing (dk_profile_enable): event pairs recorded around launches
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;  // 2 per slot
  std::vector<int> prof_kind;       // kind of each used slot
  int prof_used = 0;
  double prof_ms[DK_K_COUNT] = {};
  int64_t prof_cnt[DK_K_COUNT] = {};

  // kernels whose dynamic-LDS limit has been raised on this context's device
  // (hipFuncSetAttribute is per device): bits kAttrPlane, kAttrSlab, kAttrFermi
  unsigned lds_attr_done = 0;
  // linear solver of the Poisson and Kerker solves (dk_set_linear_solver)
  int linear_solver = DK_SOLVER_CG;
  double aar_omega = 0.6, aar_beta = 0.6;
  int aar_history = 7, aar_period = 6;
  // result of taking the address of the no-allocation scratch on this device
  hipError_t scratch_status = hipSuccess;

  // device status word and host bookkeeping
  unsigned* err_dev = nullptr;
  // spectral bounds: pinned host copies of the squaring estimates (two
  // alternating buffers) and the events that mark them ready
  double* sb_host = nullptr;
  hipEvent_t sb_ev[2] = {nullptr, nullptr};
  unsigned err_host = 0;  // same bits, raised by host-side checks within a call
  std::string last_error;
  double timings[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace dk {

enum : unsigned { kAttrPlane = 1u, kAttrSlab = 2u, kAttrFermi = 4u };

inline void flag_error(dk_ctx* c, unsigned bits) { c->err_host |= bits; }

// Bytes a workspace slice of `bytes` occupies (slices are 256-byte aligned).
inline size_t ws_slice(size_t bytes) { return (bytes + 255) & ~size_t(255); }

// Sub-allocation of the caller's workspace (256-byte aligned slices).  Every
// *_ws_bytes function returns the exact sum of the ws_slice() sizes its
// user takes; users check `ok` before launching any kernel.
struct WsCursor {
  char* base;
  size_t cap;
  size_t off = 0;
  bool ok = true;
  WsCursor(char* b, size_t c) : base(b), cap(c) {}
  template <typename T> T* take(size_t count) {
    size_t bytes = ws_slice(count * sizeof(T));
    if (off + bytes > cap) { ok = false; return nullptr; }
    T* p = (T*)(base + off);
    off += bytes;
    return p;
  }
};

// Brackets the kernel launches of its scope with a pair of HIP events when
// per-kernel timing is on (api.hip).
struct KTimer {
  dk_ctx* c;
  int slot = -1;
  KTimer(dk_ctx* ctx, int kind);
  ~KTimer();
};
void prof_flush(dk_ctx* c);

// stencil.hip
hipError_t stencil_step(dk_ctx* c, const void* yin, const void* yprev, void* yout, long ld,
                        int n_s, double alpha, double beta, double shift);
hipError_t fd_gradient_tables(dk_ctx* c);

// projectors.hip
int model_functions(int n_channels, const int* l);
hipError_t build_projector_tables(dk_ctx* c, const double* pos_dev, int n_atoms, int n_channels,
                                  const int* l, const double* rc, double cutoff_rel,
                                  double* norms_dev);

int projector_moment_stress_parts(const dk_ctx* c);
hipError_t projector_moment_stress(dk_ctx* c, const double* z, double* part, int n_part_max,
                                   int* n_part);

// scf.hip (electrostatic stress: image moments of the atom fields)
size_t es_moment_ws_bytes(const dk_ctx* c);
int es_moment_parts(const dk_ctx* c);
hipError_t es_moment_stress(dk_ctx* c, const double* rho, const double* vc, void* ws,
                            double* part);

// stress.hip
size_t electrostatic_stress_ws_bytes(const dk_ctx* c);
hipError_t electrostatic_stress(dk_ctx* c, const double* rho, const double* vc, double* sigma,
                                void* ws);
size_t stress_ws_bytes(const dk_ctx* c, int n_s);
hipError_t stress(dk_ctx* c, const void* x, long ld, int n_s, const double* ds, double* kinetic,
                  double* nonlocal, void* ws);

// nonlocal.hip
hipError_t projector_group_lists(dk_ctx* c);
size_t nonlocal_ws_bytes(const dk_ctx* c, int n_s);
// Y += alpha sum_p gamma_p chi_p (h^3 chi_p^T X) in two calls: the integrals
// of X into ws, then the scatter into Y from ws.  subspace: the product only
// shapes the filtered subspace (Chebyshev filter steps; the Rayleigh-Ritz
// projection and the forces apply H at full accuracy), and the mixed path may
// form the integrals with the two-piece split-BF16 products.
hipError_t nonlocal_integrals(dk_ctx* c, const void* x, long ld, int n_s, double alpha, void* ws,
                              bool subspace);
hipError_t nonlocal_scatter(dk_ctx* c, void* y, long ld, int n_s, void* ws);
size_t projector_integrals_ws_bytes(const dk_ctx* c, int n_s, int m_rows);
hipError_t projector_integrals(dk_ctx* c, const void* x, long ld, int n_s, const void* table,
                               int m_rows, double scale, double* out, void* ws);

// gather.hip
bool use_gather_chunks(const dk_ctx* c);
hipError_t build_gather_chunks(dk_ctx* c);
void free_gather_chunks(dk_ctx* c);
size_t gather_chunks_ws_bytes(const dk_ctx* c, int n_s);
hipError_t build_table_pieces(dk_ctx* c);
hipError_t gather_chunks(dk_ctx* c, const void* x, long ld, int n_s, double scale,
                         const double* rowscale, double* out64, float* out32, void* ws,
                         bool two_piece = false);

// linalg.hip
size_t gram_ws_bytes(const dk_ctx* c, int n_s);
hipError_t gram(dk_ctx* c, const void* x, const void* y, long ld, int n_s, bool symmetric_x,
                double scale, double* out, void* ws, bool bf16x3, int kind);
hipError_t cholesky_inverse(dk_ctx* c, double* g, int n, double* linv, double* diag);
hipError_t apply_right_upper(dk_ctx* c, const void* x, long ld, int n_s, const double* zt,
                             void* out, void* ws);
// bf16 piece planes of an FP64 matrix for the split-at-store products (mixed path)
size_t split_planes_bytes(int K, int N, int np);
long split_planes_ld(int K);
hipError_t split_planes(dk_ctx* c, const double* src, long s_k, long s_n, int K, int N, int np,
                        void* dst);
size_t spectral_ws_bytes(int n);
hipError_t spectral_bounds(dk_ctx* c, const double* hs, int n, void* ws, double* lo, double* hi,
                           int* iters);

// foe.hip
size_t foe_ws_bytes(int n_s, int n_pl);
hipError_t foe_run(dk_ctx* c, const double* hs, int n_s, double n_e, double sigma, int n_pl,
                   double* ds, double* tau_out, dk_fermi_info* info, void* ws);
hipError_t energies(dk_ctx* c, const double* tau, int n_pl, double mu, double chi, double xi,
                    double sigma, double* e_band, double* e_ent, void* ws);

// density.hip
// dk_density_noalloc's static device scratch (per GPU): 128 MiB
constexpr size_t kDensityScratchBytes = size_t(128) << 20;
// hipGetSymbolAddress of the scratch on `device` (which must be current), once
// per device; density_scratch returns that address (nullptr before the init)
hipError_t density_scratch_init(int device);
void* density_scratch(int device);
size_t density_ws_bytes(const dk_ctx* c, int n_s);
hipError_t density(dk_ctx* c, const void* x, long ld, int n_s, const double* ds, double* rho,
                   void* ws);
size_t forces_ws_bytes(const dk_ctx* c, int n_s, int n_atoms);
hipError_t forces(dk_ctx* c, const void* x, long ld, int n_s, const double* ds,
                  const double* rho, const double* gradv, int n_atoms, double* f_host, void* ws);

// scf.hip
size_t atom_tables_bytes(const dk_ctx* c, int n_atoms);
hipError_t local_fields(dk_ctx* c, const double* pos_dev, int n_atoms, double z, double rc,
                        double core_amp, double core_w2, double* tab, double* b, double* vcore);
hipError_t local_forces(dk_ctx* c, const double* tab, int n_atoms, double z, double rc,
                        double core_amp, const double* rho, const double* vc, double* f_dev);
hipError_t negate(dk_ctx* c, const double* src, double* dst);
hipError_t add_fields(dk_ctx* c, const double* a, const double* b, double* out);
size_t poisson_ws_bytes(const dk_ctx* c);
hipError_t poisson_cg(dk_ctx* c, const double* src, double* x, double tol, int max_iter,
                      void* ws, int* iters, double* relres, int* status);
size_t potential_ws_bytes();
hipError_t effective_potential(dk_ctx* c, const double* rho, const double* b, const double* vc,
                               const double* vcore, double* vxc, double* veff, void* ws,
                               double* sums);
size_t pulay_state_bytes(const dk_ctx* c, int history);
size_t kerker_pulay_state_bytes(const dk_ctx* c, int history);
hipError_t kerker_pulay_mix(dk_ctx* c, void* state, int history, int iter, int period,
                            int restart, double beta, double k0, double tol, int max_iter,
                            const double* in, const double* out, double* next, double* residual,
                            int* cg_iters, int* cg_status);
hipError_t pulay_mix(dk_ctx* c, void* state, int history, int iter, double beta,
                     const double* in, const double* out, double* next, double* residual);

hipError_t md_kick(dk_ctx* c, double* v, const double* f, double scale, int n);
hipError_t md_isokinetic_kick(dk_ctx* c, double* v, const double* f, double inv_mass, double tau,
                              int n);
hipError_t md_drift(dk_ctx* c, double* x, const double* v, double dt, int n);
hipError_t md_kinetic(dk_ctx* c, const double* v, int n, double mass, double* out_dev);

// mlp.hip
size_t mlp_params(int n_in, int hidden, int layers);
size_t desc_tables_bytes(int n_atoms, int K, int nmax);
hipError_t descriptors(dk_ctx* c, const double* pos_dev, int n_atoms, int K, const double* w_dev,
                       double* tab, float* desc);
size_t channel_stats_ws_bytes(int K);
hipError_t channel_stats(dk_ctx* c, const float* d, long n, int K, double* mean, double* inv_std,
                         void* ws);
hipError_t mlp_gather(dk_ctx* c, const float* desc, const double* rho, const int64_t* idx, int K,
                      long n_pts, const double* mean, const double* inv_std, double scale,
                      float* u, float* t);
size_t mlp_ws_bytes(int n_in, int hidden, int layers, long n_pts);
hipError_t mlp_run(dk_ctx* c, int precision, int n_in, int hidden, int layers,
                   const float* params, const float* u, const float* t, long P, float* grad,
                   double* y_out, void* ws, double* host_out);
hipError_t adam_update(dk_ctx* c, long n, float* th, float* m, float* v, const float* g, int t,
                       double lr, double b1, double b2, double eps);
size_t mlp_density_ws_bytes(int n_in, int hidden, int layers);
hipError_t mlp_density(dk_ctx* c, int precision, int n_in, int hidden, int layers,
                       const float* params, const float* desc, const double* mean,
                       const double* inv_std, double n_e, double* rho, void* ws);

// transport.hip
hipError_t time_correlation(dk_ctx* c, const double* series, long n_steps, int n_comp, int max_lag,
                            double dt, double scale, double* corr, double* integral);
hipError_t deviatoric_stress(dk_ctx* c, const double* sigma, const double* v, int n_atoms,
                             double mass, long n_steps, double* out);

// small utilities (linalg.hip)
hipError_t copy_block(dk_ctx* c, const void* src, void* dst, long ld, int n_s);
hipError_t check_finite(dk_ctx* c, const double* p, long n);

}  // namespace dk
