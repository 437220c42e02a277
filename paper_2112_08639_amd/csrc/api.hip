// C ABI of libdk (declarations and contracts in include/dk.h).
#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "ctx.h"

using namespace dk;

namespace {

enum TimerSlot { kTFilter = 0, kTOrth, kTProject, kTBounds, kTDk, kTDensity, kTEnergy, kTForces };

dk_status fail(dk_ctx* c, dk_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
dk_status fail(dk_ctx* c, dk_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->last_error = buf;
  }
  return s;
}

dk_status hip_fail(dk_ctx* c, hipError_t e, const char* where) {
  return fail(c, DK_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define DK_HIP(c, call)                                          \
  do {                                                           \
    hipError_t e_ = (call);                                      \
    if (e_ != hipSuccess) return hip_fail((c), e_, #call);       \
  } while (0)

struct Timed {
  dk_ctx* c;
  int slot;
  Timed(dk_ctx* c_, int s) : c(c_), slot(s) { hipEventRecord(c->ev0, c->stream); }
  ~Timed() {}
  void stop() {
    hipEventRecord(c->ev1, c->stream);
    hipEventSynchronize(c->ev1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, c->ev0, c->ev1);
    c->timings[slot] = ms;
  }
};

// Synchronise, then turn the device status word into a dk_status.
dk_status finish(dk_ctx* c, const char* what) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, what);
  unsigned flags = 0;
  e = hipMemcpy(&flags, c->err_dev, sizeof flags, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, what);
  flags |= c->err_host;
  c->err_host = 0;
  if (flags) {
    unsigned zero = 0;
    hipMemcpy(c->err_dev, &zero, sizeof zero, hipMemcpyHostToDevice);
    if (flags & kErrNotSpd) return fail(c, DK_ERR_NOT_SPD, "%s: Gram matrix not positive definite", what);
    if (flags & kErrFermi) return fail(c, DK_ERR_FERMI, "%s: electron count not bracketed", what);
    if (flags & kErrNonFinite) return fail(c, DK_ERR_NONFINITE, "%s: non-finite value", what);
    if (flags & kErrConvergence) return fail(c, DK_ERR_CONVERGENCE, "%s: spectral bounds did not converge", what);
    if (flags & kErrDegree)
      return fail(c, DK_ERR_CONVERGENCE, "%s: no expansion degree up to %d meets the coefficient tail %g", what, kTailCap, kTailTol);
  }
  c->last_error.clear();
  return DK_OK;
}

size_t elem_size(const dk_ctx* c) { return c->precision == DK_PREC_FP64 ? 8 : 4; }

dk_status check_block(dk_ctx* c, const void* X, int64_t ld, int n_s, const char* what) {
  if (!c) return DK_ERR_ARG;
  if (!X) return fail(c, DK_ERR_ARG, "%s: null block pointer", what);
  if (n_s <= 0) return fail(c, DK_ERR_ARG, "%s: n_s must be positive (got %d)", what, n_s);
  if (ld < c->ngrid) return fail(c, DK_ERR_ARG, "%s: ld %lld < N_grid %ld", what, (long long)ld, c->ngrid);
  if (!c->have_potential) return fail(c, DK_ERR_STATE, "%s: dk_set_potential has not been called", what);
  return DK_OK;
}

dk_status need_ws(dk_ctx* c, size_t bytes, const char* what) {
  if (!c->ws || c->ws_bytes < bytes)
    return fail(c, DK_ERR_ALLOC, "%s: workspace of %zu bytes needed, %zu set (see dk_workspace_bytes)",
                what, bytes, c->ws_bytes);
  return DK_OK;
}

size_t block_bytes(const dk_ctx* c, int n_s, int64_t ld) {
  return ws_slice((size_t)ld * n_s * elem_size(c));
}

// exact workspace of each call: the sum of the slices it takes
size_t ws_filter(const dk_ctx* c, int n_s, int64_t ld) {
  return block_bytes(c, n_s, ld) + ws_slice(nonlocal_ws_bytes(c, n_s));
}
size_t ws_orth(const dk_ctx* c, int n_s, int64_t ld) {
  return block_bytes(c, n_s, ld) + 2 * ws_slice((size_t)n_s * n_s * 8) +
         ws_slice((size_t)n_s * 8) + ws_slice(gram_ws_bytes(c, n_s));
}
size_t ws_project_aux(const dk_ctx* c, int n_s) {
  return std::max(gram_ws_bytes(c, n_s), nonlocal_ws_bytes(c, n_s));
}
size_t ws_project(const dk_ctx* c, int n_s, int64_t ld) {
  return block_bytes(c, n_s, ld) + ws_slice(ws_project_aux(c, n_s));
}
size_t ws_density(const dk_ctx* c, int n_s) { return density_ws_bytes(c, n_s); }
size_t ws_scf(const dk_ctx* c) {
  const int na = c->n_local_atoms > 0 ? c->n_local_atoms : 1;
  return ws_slice(poisson_ws_bytes(c)) + ws_slice(c->ngrid * sizeof(double)) +
         ws_slice(potential_ws_bytes()) + ws_slice(3 * (size_t)na * sizeof(double));
}

void free_atoms(dk_ctx* c) {
  hipFree(c->pos_dev); c->pos_dev = nullptr;
  hipFree(c->atom_tab); c->atom_tab = nullptr;
  hipFree(c->b_dev); c->b_dev = nullptr;
  hipFree(c->vcore_dev); c->vcore_dev = nullptr;
  c->n_local_atoms = 0;
}

}  // namespace

namespace dk {

KTimer::KTimer(dk_ctx* ctx, int kind) : c(ctx) {
  if (!c->prof_on) return;
  if (c->prof_used * 2 + 2 > (int)c->prof_ev.size()) prof_flush(c);
  slot = c->prof_used++;
  c->prof_kind[slot] = kind;
  hipEventRecord(c->prof_ev[2 * slot], c->stream);
}

KTimer::~KTimer() {
  if (slot >= 0) hipEventRecord(c->prof_ev[2 * slot + 1], c->stream);
}

void prof_flush(dk_ctx* c) {
  if (c->prof_used == 0) return;
  hipEventSynchronize(c->prof_ev[2 * c->prof_used - 1]);
  for (int i = 0; i < c->prof_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->prof_ev[2 * i], c->prof_ev[2 * i + 1]) == hipSuccess) {
      c->prof_ms[c->prof_kind[i]] += ms;
      c->prof_cnt[c->prof_kind[i]] += 1;
    }
  }
  c->prof_used = 0;
}

}  // namespace dk

extern "C" {

int dk_version(void) { return 100; }

const char* dk_status_name(int s) {
  switch (s) {
    case DK_OK: return "DK_OK";
    case DK_ERR_ARG: return "DK_ERR_ARG";
    case DK_ERR_DEVICE: return "DK_ERR_DEVICE";
    case DK_ERR_ALLOC: return "DK_ERR_ALLOC";
    case DK_ERR_NOT_SPD: return "DK_ERR_NOT_SPD";
    case DK_ERR_FERMI: return "DK_ERR_FERMI";
    case DK_ERR_NONFINITE: return "DK_ERR_NONFINITE";
    case DK_ERR_STATE: return "DK_ERR_STATE";
    case DK_ERR_CONVERGENCE: return "DK_ERR_CONVERGENCE";
    default: return "DK_ERR_UNKNOWN";
  }
}

dk_status dk_create(dk_ctx** out, int nx, int ny, int nz, double lx, double ly, double lz,
                    int precision, int device, void* stream) {
  if (!out) return DK_ERR_ARG;
  *out = nullptr;
  if (nx < 7 || ny < 7 || nz < 7 || nx > 1024) return DK_ERR_ARG;
  if (!(lx > 0) || !(ly > 0) || !(lz > 0)) return DK_ERR_ARG;
  if (precision != DK_PREC_FP64 && precision != DK_PREC_MIXED) return DK_ERR_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return DK_ERR_DEVICE;
  if (device < 0 || device >= ndev) return DK_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return DK_ERR_DEVICE;
  dk_ctx* c = new (std::nothrow) dk_ctx();
  if (!c) return DK_ERR_ALLOC;
  c->nx = nx; c->ny = ny; c->nz = nz;
  c->ngrid = (long)nx * ny * nz;
  c->lx = lx; c->ly = ly; c->lz = lz;
  c->hx = lx / nx; c->hy = ly / ny; c->hz = lz / nz;
  c->dv = c->hx * c->hy * c->hz;
  c->precision = precision;
  c->device = device;
  c->stream = (hipStream_t)stream;
  if (hipMalloc(&c->err_dev, 256) != hipSuccess) { delete c; return DK_ERR_ALLOC; }
  hipMemset(c->err_dev, 0, 256);
  hipEventCreate(&c->ev0);
  hipEventCreate(&c->ev1);
  // device address of the no-allocation scratch, once per device (with the
  // device current); a failure only disables dk_density_noalloc
  c->scratch_status = density_scratch_init(device);
  *out = c;
  return DK_OK;
}

static void free_tables(dk_ctx* c) {
  hipFree(c->chi64); c->chi64 = nullptr;
  hipFree(c->chi32); c->chi32 = nullptr;
  hipFree(c->chi_pieces); c->chi_pieces = nullptr;
  c->chi_pieces_bytes = 0;
  c->dchi64 = nullptr;  // part of the chi64 allocation
  hipFree(c->gamma_dev); c->gamma_dev = nullptr;
  hipFree(c->atom_dev); c->atom_dev = nullptr;
  hipFree(c->mask_t); c->mask_t = nullptr;
  hipFree(c->klist); c->klist = nullptr;
  hipFree(c->kcount); c->kcount = nullptr;
  free_gather_chunks(c);
  c->n_groups = 0;
  c->n_proj = 0;
  c->model_channels = 0;
}

dk_status dk_destroy(dk_ctx* c) {
  if (!c) return DK_OK;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream); else hipDeviceSynchronize();
  if (c->sb_host) hipHostFree(c->sb_host);
  for (hipEvent_t& ev : c->sb_ev)
    if (ev) hipEventDestroy(ev);
  free_tables(c);
  free_atoms(c);
  hipFree(c->proj_aux);
  hipFree(c->veff64);
  hipFree(c->veff32);
  hipFree(c->err_dev);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  delete c;
  return DK_OK;
}

const char* dk_last_error(const dk_ctx* c) { return c ? c->last_error.c_str() : "null context"; }

namespace {
__global__ void to_f32_kernel(const double* __restrict__ s, float* __restrict__ d, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    d[e] = (float)s[e];
}
}  // namespace

dk_status dk_set_potential(dk_ctx* c, const double* veff) {
  if (!c) return DK_ERR_ARG;
  if (!veff) return fail(c, DK_ERR_ARG, "dk_set_potential: null pointer");
  hipSetDevice(c->device);
  if (!c->veff64) DK_HIP(c, hipMalloc(&c->veff64, c->ngrid * sizeof(double)));
  if (!c->veff32) DK_HIP(c, hipMalloc(&c->veff32, c->ngrid * sizeof(float)));
  DK_HIP(c, hipMemcpyAsync(c->veff64, veff, c->ngrid * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  DK_HIP(c, check_finite(c, c->veff64, c->ngrid));
  long b = (c->ngrid + 255) / 256; if (b > 4096) b = 4096;
  hipLaunchKernelGGL(to_f32_kernel, dim3((int)b), dim3(256), 0, c->stream, c->veff64, c->veff32, c->ngrid);
  std::vector<double> h(c->ngrid);
  DK_HIP(c, hipMemcpyAsync(h.data(), c->veff64, c->ngrid * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  dk_status s = finish(c, "dk_set_potential");
  if (s != DK_OK) return s;
  c->vmax = *std::max_element(h.begin(), h.end());
  c->have_potential = true;
  return DK_OK;
}

dk_status dk_set_projectors(dk_ctx* c, int n_proj, int n_atoms, const int64_t* offsets,
                            const int32_t* indices, const double* values, const double* gamma,
                            const int32_t* atom) {
  if (!c) return DK_ERR_ARG;
  if (n_proj < 0 || n_atoms < 0) return fail(c, DK_ERR_ARG, "dk_set_projectors: negative count");
  hipSetDevice(c->device);
  free_tables(c);
  c->n_atoms = n_atoms;
  c->nl_bound = 0.0;
  c->gamma_h.clear();
  c->atom_h.clear();
  if (n_proj == 0) return DK_OK;
  if (!offsets || !indices || !values || !gamma || !atom)
    return fail(c, DK_ERR_ARG, "dk_set_projectors: null table pointer");
  if (offsets[0] != 0) return fail(c, DK_ERR_ARG, "dk_set_projectors: offsets[0] must be 0");
  const long ng = c->ngrid;
  std::vector<double> dense((size_t)ng * n_proj, 0.0);
  for (int p = 0; p < n_proj; ++p) {
    if (offsets[p + 1] < offsets[p]) return fail(c, DK_ERR_ARG, "dk_set_projectors: offsets not monotone at %d", p);
    if (atom[p] < 0 || atom[p] >= n_atoms) return fail(c, DK_ERR_ARG, "dk_set_projectors: atom[%d] out of range", p);
    if (!std::isfinite(gamma[p])) return fail(c, DK_ERR_NONFINITE, "dk_set_projectors: gamma[%d] not finite", p);
    double nrm = 0.0;
    for (int64_t e = offsets[p]; e < offsets[p + 1]; ++e) {
      const int32_t ix = indices[e];
      if (ix < 0 || ix >= ng) return fail(c, DK_ERR_ARG, "dk_set_projectors: index %d out of range", ix);
      if (!std::isfinite(values[e])) return fail(c, DK_ERR_NONFINITE, "dk_set_projectors: value not finite");
      dense[(size_t)p * ng + ix] = values[e];
      nrm += values[e] * values[e];
    }
    if (gamma[p] > 0) c->nl_bound += gamma[p] * c->dv * nrm;
    c->gamma_h.push_back(gamma[p]);
    c->atom_h.push_back(atom[p]);
  }
  // block masks
  const long gblocks = (ng + 63) / 64;
  const int ptiles = (n_proj + 63) / 64;
  std::vector<uint8_t> mt((size_t)ptiles * gblocks, 0);
  for (int p = 0; p < n_proj; ++p)
    for (long x = 0; x < ng; ++x)
      if (dense[(size_t)p * ng + x] != 0.0) {
        mt[(size_t)(p / 64) * gblocks + x / 64] = 1;
      }
  c->mask_t_stride = gblocks;
  std::vector<float> dense32(dense.begin(), dense.end());
  // chi and its three finite-difference gradients are one N_grid x 4 n_proj
  // table, so the force contractions read the block once
  DK_HIP(c, hipMalloc(&c->chi64, 4 * dense.size() * sizeof(double)));
  c->dchi64 = c->chi64 + dense.size();
  if (c->precision == DK_PREC_MIXED) DK_HIP(c, hipMalloc(&c->chi32, dense.size() * sizeof(float)));
  DK_HIP(c, hipMalloc(&c->gamma_dev, n_proj * sizeof(double)));
  DK_HIP(c, hipMalloc(&c->atom_dev, n_proj * sizeof(int)));
  DK_HIP(c, hipMalloc(&c->mask_t, mt.size()));
  DK_HIP(c, hipMemcpy(c->chi64, dense.data(), dense.size() * sizeof(double), hipMemcpyHostToDevice));
  if (c->chi32) DK_HIP(c, hipMemcpy(c->chi32, dense32.data(), dense32.size() * sizeof(float), hipMemcpyHostToDevice));
  DK_HIP(c, hipMemcpy(c->gamma_dev, c->gamma_h.data(), n_proj * sizeof(double), hipMemcpyHostToDevice));
  DK_HIP(c, hipMemcpy(c->atom_dev, c->atom_h.data(), n_proj * sizeof(int), hipMemcpyHostToDevice));
  DK_HIP(c, hipMemcpy(c->mask_t, mt.data(), mt.size(), hipMemcpyHostToDevice));
  c->n_proj = n_proj;
  DK_HIP(c, fd_gradient_tables(c));
  DK_HIP(c, projector_group_lists(c));
  DK_HIP(c, build_gather_chunks(c));
  DK_HIP(c, build_table_pieces(c));
  return finish(c, "dk_set_projectors");
}

dk_status dk_set_projector_model(dk_ctx* c, int n_atoms, const double* pos, int n_channels,
                                 const int32_t* l, const double* rc, const double* gamma,
                                 double cutoff_rel) {
  if (!c) return DK_ERR_ARG;
  if (n_atoms < 0) return fail(c, DK_ERR_ARG, "dk_set_projector_model: negative atom count");
  if (n_channels < 1 || n_channels > DK_PROJ_MAX_CHANNELS)
    return fail(c, DK_ERR_ARG, "dk_set_projector_model: need 1 <= n_channels <= %d", DK_PROJ_MAX_CHANNELS);
  if (!l || !rc || !gamma || (n_atoms > 0 && !pos))
    return fail(c, DK_ERR_ARG, "dk_set_projector_model: null pointer");
  for (int k = 0; k < n_channels; ++k) {
    if (l[k] != 0 && l[k] != 1) return fail(c, DK_ERR_ARG, "dk_set_projector_model: l[%d] must be 0 or 1", k);
    if (!(rc[k] > 0) || !std::isfinite(rc[k])) return fail(c, DK_ERR_ARG, "dk_set_projector_model: rc[%d] must be finite and > 0", k);
    if (!std::isfinite(gamma[k])) return fail(c, DK_ERR_NONFINITE, "dk_set_projector_model: gamma[%d] not finite", k);
  }
  if (!(cutoff_rel > 0 && cutoff_rel < 1)) return fail(c, DK_ERR_ARG, "dk_set_projector_model: need 0 < cutoff_rel < 1");
  for (int i = 0; i < 3 * n_atoms; ++i)
    if (!std::isfinite(pos[i])) return fail(c, DK_ERR_NONFINITE, "dk_set_projector_model: position %d not finite", i);
  hipSetDevice(c->device);
  const int per_atom = model_functions(n_channels, l);
  const long n_proj_l = (long)n_atoms * per_atom;
  if (n_proj_l > (1L << 24)) return fail(c, DK_ERR_ARG, "dk_set_projector_model: %ld projectors exceed 2^24", n_proj_l);
  const int n_proj = (int)n_proj_l;
  const long ng = c->ngrid;
  if (n_proj == 0) {
    free_tables(c);
    c->n_atoms = n_atoms;
    c->nl_bound = 0.0;
    c->gamma_h.clear();
    c->atom_h.clear();
    return DK_OK;
  }
  const long gblocks = (ng + 63) / 64;
  const int ptiles = (n_proj + 63) / 64;
  const size_t table = (size_t)ng * n_proj;
  // keep the tables of the previous call when the sizes match (an ionic step)
  if (n_proj != c->n_proj || !c->chi64 || (c->precision == DK_PREC_MIXED) != (c->chi32 != nullptr)) {
    free_tables(c);
    DK_HIP(c, hipMalloc(&c->chi64, 4 * table * sizeof(double)));
    c->dchi64 = c->chi64 + table;
    if (c->precision == DK_PREC_MIXED) DK_HIP(c, hipMalloc(&c->chi32, table * sizeof(float)));
    DK_HIP(c, hipMalloc(&c->gamma_dev, n_proj * sizeof(double)));
    DK_HIP(c, hipMalloc(&c->atom_dev, n_proj * sizeof(int)));
    DK_HIP(c, hipMalloc(&c->mask_t, (size_t)ptiles * gblocks));
  }
  const size_t aux = 3 * (size_t)n_atoms + n_proj;
  if (aux > c->proj_aux_len) {
    hipFree(c->proj_aux);
    c->proj_aux = nullptr;
    c->proj_aux_len = 0;
    DK_HIP(c, hipMalloc(&c->proj_aux, aux * sizeof(double)));
    c->proj_aux_len = aux;
  }
  c->n_atoms = n_atoms;
  c->gamma_h.clear();
  c->atom_h.clear();
  c->model_channels = n_channels;
  for (int k = 0; k < n_channels; ++k) {
    c->model_l[k] = l[k];
    c->model_rc[k] = rc[k];
  }
  c->model_cutoff_rel = cutoff_rel;
  for (int a = 0; a < n_atoms; ++a)
    for (int k = 0; k < n_channels; ++k)
      for (int m = 0; m < (l[k] == 0 ? 1 : 3); ++m) {
        c->gamma_h.push_back(gamma[k]);
        c->atom_h.push_back(a);
      }
  c->mask_t_stride = gblocks;
  double* pos_dev = c->proj_aux;
  double* norms_dev = c->proj_aux + 3 * (size_t)n_atoms;
  DK_HIP(c, hipMemcpyAsync(pos_dev, pos, 3 * (size_t)n_atoms * sizeof(double), hipMemcpyHostToDevice, c->stream));
  DK_HIP(c, hipMemcpyAsync(c->gamma_dev, c->gamma_h.data(), n_proj * sizeof(double), hipMemcpyHostToDevice, c->stream));
  DK_HIP(c, hipMemcpyAsync(c->atom_dev, c->atom_h.data(), n_proj * sizeof(int), hipMemcpyHostToDevice, c->stream));
  DK_HIP(c, build_projector_tables(c, pos_dev, n_atoms, n_channels, l, rc, cutoff_rel, norms_dev));
  c->n_proj = n_proj;
  DK_HIP(c, fd_gradient_tables(c));
  DK_HIP(c, projector_group_lists(c));
  DK_HIP(c, build_gather_chunks(c));
  DK_HIP(c, build_table_pieces(c));
  std::vector<double> nrm(n_proj);
  DK_HIP(c, hipMemcpyAsync(nrm.data(), norms_dev, n_proj * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  dk_status s = finish(c, "dk_set_projector_model");
  if (s != DK_OK) return s;
  c->nl_bound = 0.0;
  for (int p = 0; p < n_proj; ++p)
    if (c->gamma_h[p] > 0) c->nl_bound += c->gamma_h[p] * c->dv * nrm[p];
  return DK_OK;
}

dk_status dk_spectrum_upper_bound(dk_ctx* c, double* b) {
  if (!c || !b) return c ? fail(c, DK_ERR_ARG, "dk_spectrum_upper_bound: null output") : DK_ERR_ARG;
  if (!c->have_potential) return fail(c, DK_ERR_STATE, "dk_spectrum_upper_bound: no potential");
  // kinetic symbol at the zone corner: s(pi) = -w_0 - 2 sum_k (-1)^k w_k
  static const double w[7] = {-5369.0 / 1800.0, 12.0 / 7.0, -15.0 / 56.0, 10.0 / 189.0,
                              -1.0 / 112.0, 2.0 / 1925.0, -1.0 / 16632.0};
  double s = -w[0];
  for (int k = 1; k <= 6; ++k) s -= 2.0 * ((k % 2) ? -1.0 : 1.0) * w[k];
  const double kin = 0.5 * s * (1.0 / (c->hx * c->hx) + 1.0 / (c->hy * c->hy) + 1.0 / (c->hz * c->hz));
  *b = kin + c->vmax + c->nl_bound;
  return DK_OK;
}

dk_status dk_workspace_bytes(const dk_ctx* c, int n_s, int64_t ld, int n_pl, size_t* bytes) {
  if (!c || !bytes || n_s <= 0 || ld < c->ngrid || n_pl < 0) return DK_ERR_ARG;
  size_t b = ws_filter(c, n_s, ld);
  b = std::max(b, ws_orth(c, n_s, ld));
  b = std::max(b, ws_project(c, n_s, ld));
  b = std::max(b, foe_ws_bytes(n_s, n_pl));
  b = std::max(b, ws_density(c, n_s));
  b = std::max(b, forces_ws_bytes(c, n_s, c->n_atoms));
  b = std::max(b, stress_ws_bytes(c, n_s));
  b = std::max(b, electrostatic_stress_ws_bytes(c));
  b = std::max(b, spectral_ws_bytes(n_s));
  b = std::max(b, ws_scf(c));
  *bytes = b + 4096;
  return DK_OK;
}

dk_status dk_set_workspace(dk_ctx* c, void* p, size_t bytes) {
  if (!c) return DK_ERR_ARG;
  if (p && ((uintptr_t)p % 256) != 0) return fail(c, DK_ERR_ARG, "dk_set_workspace: pointer not 256-byte aligned");
  c->ws = (char*)p;
  c->ws_bytes = p ? bytes : 0;
  return DK_OK;
}

dk_status dk_apply_h(dk_ctx* c, const void* X, void* Y, int64_t ld, int n_s) {
  dk_status s = check_block(c, X, ld, n_s, "dk_apply_h");
  if (s != DK_OK) return s;
  if (!Y) return fail(c, DK_ERR_ARG, "dk_apply_h: null output");
  if ((s = need_ws(c, nonlocal_ws_bytes(c, n_s), "dk_apply_h")) != DK_OK) return s;
  hipSetDevice(c->device);
  // integrals first, as in the filter: both reads of X come together
  DK_HIP(c, nonlocal_integrals(c, X, ld, n_s, 1.0, c->ws, false));
  DK_HIP(c, stencil_step(c, X, nullptr, Y, ld, n_s, 1.0, 0.0, 0.0));
  DK_HIP(c, nonlocal_scatter(c, Y, ld, n_s, c->ws));
  return finish(c, "dk_apply_h");
}

dk_status dk_filter(dk_ctx* c, void* X, int64_t ld, int n_s, int degree, double a, double b,
                    double a0) {
  dk_status s = check_block(c, X, ld, n_s, "dk_filter");
  if (s != DK_OK) return s;
  if (degree < 1) return fail(c, DK_ERR_ARG, "dk_filter: degree must be >= 1");
  if (!(a0 < a && a < b) || !std::isfinite(a0) || !std::isfinite(b))
    return fail(c, DK_ERR_ARG, "dk_filter: need a0 < a < b (got %g, %g, %g)", a0, a, b);
  if ((s = need_ws(c, ws_filter(c, n_s, ld), "dk_filter")) != DK_OK) return s;
  hipSetDevice(c->device);
  Timed tm(c, kTFilter);
  WsCursor cur(c->ws, c->ws_bytes);
  void* W = cur.take<char>((size_t)ld * n_s * elem_size(c));
  void* nl = cur.take<char>(nonlocal_ws_bytes(c, n_s));
  if (!cur.ok) return fail(c, DK_ERR_ALLOC, "dk_filter: workspace layout overflow");
  // Y_0 = X (buffer P), Y_1 -> buffer Q, Y_{k+1} overwrites Y_{k-1} in place.
  // Each step forms the projector integrals of Y_k first, then the stencil
  // reads Y_k again and writes the local part of Y_{k+1}, then the scatter adds
  // the nonlocal part: the two reads of Y_k follow the previous step's scatter,
  // which has just written it, and find much of it still in the 256 MB
  // last-level cache (al32 filter 10.25 -> 9.84 ms per step against the stencil
  // first).
  const double e = 0.5 * (b - a), cc = 0.5 * (b + a);
  const double s1 = e / (a0 - cc);
  double sk = s1;
  void* P = X;
  void* Q = W;
  DK_HIP(c, nonlocal_integrals(c, P, ld, n_s, s1 / e, nl, true));
  DK_HIP(c, stencil_step(c, P, nullptr, Q, ld, n_s, s1 / e, 0.0, cc));
  DK_HIP(c, nonlocal_scatter(c, Q, ld, n_s, nl));
  for (int k = 1; k < degree; ++k) {
    const double sn = 1.0 / (2.0 / s1 - sk);
    const double al = 2.0 * sn / e, be = -sk * sn;
    // new iterate into P (holds Y_{k-1}), from Y_k in Q
    DK_HIP(c, nonlocal_integrals(c, Q, ld, n_s, al, nl, true));
    DK_HIP(c, stencil_step(c, Q, P, P, ld, n_s, al, be, cc));
    DK_HIP(c, nonlocal_scatter(c, P, ld, n_s, nl));
    std::swap(P, Q);
    sk = sn;
  }
  // the result is in Q
  if (Q != X) {
    KTimer kt(c, DK_K_OTHER);
    DK_HIP(c, copy_block(c, Q, X, ld, n_s));
  }
  tm.stop();
  return finish(c, "dk_filter");
}

dk_status dk_orthonormalize(dk_ctx* c, void* X, int64_t ld, int n_s) {
  dk_status s = check_block(c, X, ld, n_s, "dk_orthonormalize");
  if (s != DK_OK) return s;
  if (n_s > c->ngrid) return fail(c, DK_ERR_ARG, "dk_orthonormalize: n_s > N_grid");
  if ((s = need_ws(c, ws_orth(c, n_s, ld), "dk_orthonormalize")) != DK_OK) return s;
  hipSetDevice(c->device);
  Timed tm(c, kTOrth);
  WsCursor cur(c->ws, c->ws_bytes);
  void* W = cur.take<char>((size_t)ld * n_s * elem_size(c));
  double* G = cur.take<double>((size_t)n_s * n_s);
  double* Li = cur.take<double>((size_t)n_s * n_s);
  double* dg = cur.take<double>((size_t)n_s);
  void* gws = cur.take<char>(gram_ws_bytes(c, n_s));
  if (!cur.ok) return fail(c, DK_ERR_ALLOC, "dk_orthonormalize: workspace layout overflow");
  void* src = X;
  void* dst = W;
  for (int pass = 0; pass < 2; ++pass) {
    DK_HIP(c, gram(c, src, src, ld, n_s, true, c->dv, G, gws, false, DK_K_GRAM));
    DK_HIP(c, check_finite(c, G, (long)n_s * n_s));
    {
      KTimer kt(c, DK_K_CHOLESKY);
      DK_HIP(c, cholesky_inverse(c, G, n_s, Li, dg));
    }
    {
      KTimer kt(c, DK_K_ORTH_APPLY);
      DK_HIP(c, apply_right_upper(c, src, ld, n_s, Li, dst, gws));
    }
    std::swap(src, dst);
  }
  tm.stop();
  return finish(c, "dk_orthonormalize");
}

dk_status dk_project(dk_ctx* c, const void* X, int64_t ld, int n_s, double* hs) {
  dk_status s = check_block(c, X, ld, n_s, "dk_project");
  if (s != DK_OK) return s;
  if (!hs) return fail(c, DK_ERR_ARG, "dk_project: null output");
  if ((s = need_ws(c, ws_project(c, n_s, ld), "dk_project")) != DK_OK) return s;
  hipSetDevice(c->device);
  Timed tm(c, kTProject);
  WsCursor cur(c->ws, c->ws_bytes);
  void* HX = cur.take<char>((size_t)ld * n_s * elem_size(c));
  void* aux = cur.take<char>(ws_project_aux(c, n_s));
  if (!cur.ok) return fail(c, DK_ERR_ALLOC, "dk_project: workspace layout overflow");
  // integrals first, as in the filter: both reads of X come together
  DK_HIP(c, nonlocal_integrals(c, X, ld, n_s, 1.0, aux, false));
  DK_HIP(c, stencil_step(c, X, nullptr, HX, ld, n_s, 1.0, 0.0, 0.0));
  DK_HIP(c, nonlocal_scatter(c, HX, ld, n_s, aux));
  DK_HIP(c, gram(c, X, HX, ld, n_s, false, c->dv, hs, aux, true, DK_K_PROJECT));
  tm.stop();
  return finish(c, "dk_project");
}

dk_status dk_spectral_bounds(dk_ctx* c, const double* hs, int n_s, double* lo, double* hi, int* iters) {
  if (!c) return DK_ERR_ARG;
  if (!hs || !lo || !hi || n_s <= 0) return fail(c, DK_ERR_ARG, "dk_spectral_bounds: bad argument");
  dk_status s;
  if ((s = need_ws(c, spectral_ws_bytes(n_s), "dk_spectral_bounds")) != DK_OK) return s;
  hipSetDevice(c->device);
  Timed tm(c, kTBounds);
  {
    KTimer kt(c, DK_K_BOUNDS);
    DK_HIP(c, spectral_bounds(c, hs, n_s, c->ws, lo, hi, iters));
  }
  tm.stop();
  return finish(c, "dk_spectral_bounds");
}

dk_status dk_density_kernel(dk_ctx* c, const double* hs, int n_s, double n_e, double sigma, int n_pl,
                            double* ds, double* tau, dk_fermi_info* info) {
  if (!c) return DK_ERR_ARG;
  if (!hs || !ds || !info) return fail(c, DK_ERR_ARG, "dk_density_kernel: null pointer");
  if (n_s <= 0 || n_pl < 0) return fail(c, DK_ERR_ARG, "dk_density_kernel: need n_s > 0, n_pl >= 0");
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(c, DK_ERR_ARG, "dk_density_kernel: sigma must be > 0");
  if (!(n_e > 0) || !(n_e < 2.0 * n_s)) return fail(c, DK_ERR_FERMI, "dk_density_kernel: need 0 < N_e < 2 N_s");
  dk_status s;
  if ((s = need_ws(c, foe_ws_bytes(n_s, n_pl), "dk_density_kernel")) != DK_OK) return s;
  hipSetDevice(c->device);
  Timed tm(c, kTDk);
  DK_HIP(c, foe_run(c, hs, n_s, n_e, sigma, n_pl, ds, tau, info, c->ws));
  tm.stop();
  return finish(c, "dk_density_kernel");
}

dk_status dk_density(dk_ctx* c, const void* X, int64_t ld, int n_s, const double* ds, double* rho) {
  dk_status s = check_block(c, X, ld, n_s, "dk_density");
  if (s != DK_OK) return s;
  if (!ds || !rho) return fail(c, DK_ERR_ARG, "dk_density: null pointer");
  if ((s = need_ws(c, ws_density(c, n_s), "dk_density")) != DK_OK) return s;
  hipSetDevice(c->device);
  Timed tm(c, kTDensity);
  {
    KTimer kt(c, DK_K_DENSITY);
    DK_HIP(c, density(c, X, ld, n_s, ds, rho, c->ws));
  }
  tm.stop();
  return finish(c, "dk_density");
}

dk_status dk_density_noalloc(dk_ctx* c, const void* X, int64_t ld, int n_s, const double* ds,
                             double* rho) {
  dk_status s = check_block(c, X, ld, n_s, "dk_density_noalloc");
  if (s != DK_OK) return s;
  if (!ds || !rho) return fail(c, DK_ERR_ARG, "dk_density_noalloc: null pointer");
  const size_t need = ws_density(c, n_s);
  if (need > kDensityScratchBytes)
    return fail(c, DK_ERR_ARG,
                "dk_density_noalloc: N_grid %ld with n_s %d needs %zu bytes of scratch, more than "
                "the %zu of the static scratch (use dk_density with a workspace)",
                c->ngrid, n_s, need, kDensityScratchBytes);
  if (c->scratch_status != hipSuccess)
    return hip_fail(c, c->scratch_status, "dk_density_noalloc: scratch address");
  void* ptr = density_scratch(c->device);
  if (!ptr) return fail(c, DK_ERR_DEVICE, "dk_density_noalloc: no scratch on device %d", c->device);
  hipSetDevice(c->device);
  Timed tm(c, kTDensity);
  // no per-kernel timer: its event pool may grow
  DK_HIP(c, density(c, X, ld, n_s, ds, rho, ptr));
  tm.stop();
  return finish(c, "dk_density_noalloc");
}

dk_status dk_energy(dk_ctx* c, const double* tau, int n_pl, double mu, double chi, double xi,
                    double sigma, double* e_band, double* e_ent) {
  if (!c) return DK_ERR_ARG;
  if (!tau || !e_band || !e_ent || n_pl < 1) return fail(c, DK_ERR_ARG, "dk_energy: bad argument");
  if (!(sigma > 0) || !(xi > 0)) return fail(c, DK_ERR_ARG, "dk_energy: need sigma > 0, xi > 0");
  dk_status s;
  if ((s = need_ws(c, foe_ws_bytes(1, n_pl), "dk_energy")) != DK_OK) return s;
  hipSetDevice(c->device);
  Timed tm(c, kTEnergy);
  {
    KTimer kt(c, DK_K_FERMI);
    DK_HIP(c, energies(c, tau, n_pl, mu, chi, xi, sigma, e_band, e_ent, c->ws));
  }
  tm.stop();
  return finish(c, "dk_energy");
}

dk_status dk_forces(dk_ctx* c, const void* X, int64_t ld, int n_s, const double* ds, const double* rho,
                    const double* gradv, int n_atoms, double* f) {
  dk_status s = check_block(c, X, ld, n_s, "dk_forces");
  if (s != DK_OK) return s;
  if (!ds || !f || n_atoms <= 0) return fail(c, DK_ERR_ARG, "dk_forces: bad argument");
  if (gradv && !rho) return fail(c, DK_ERR_ARG, "dk_forces: local force needs rho");
  if (c->n_proj > 0 && n_atoms != c->n_atoms)
    return fail(c, DK_ERR_ARG, "dk_forces: n_atoms %d differs from the projector tables' %d", n_atoms, c->n_atoms);
  if ((s = need_ws(c, forces_ws_bytes(c, n_s, n_atoms), "dk_forces")) != DK_OK) return s;
  hipSetDevice(c->device);
  Timed tm(c, kTForces);
  {
    KTimer kt(c, DK_K_FORCES);
    DK_HIP(c, forces(c, X, ld, n_s, ds, rho, gradv, n_atoms, f, c->ws));
  }
  tm.stop();
  return finish(c, "dk_forces");
}

dk_status dk_stress(dk_ctx* c, const void* X, int64_t ld, int n_s, const double* ds,
                    double* kinetic, double* nonlocal) {
  dk_status s = check_block(c, X, ld, n_s, "dk_stress");
  if (s != DK_OK) return s;
  if (!ds || !kinetic || !nonlocal) return fail(c, DK_ERR_ARG, "dk_stress: null argument");
  if (c->n_proj > 0 && c->model_channels == 0)
    return fail(c, DK_ERR_STATE, "dk_stress: nonlocal stress needs tables from dk_set_projector_model");
  if ((s = need_ws(c, stress_ws_bytes(c, n_s), "dk_stress")) != DK_OK) return s;
  hipSetDevice(c->device);
  {
    KTimer kt(c, DK_K_STRESS);
    DK_HIP(c, stress(c, X, ld, n_s, ds, kinetic, nonlocal, c->ws));
  }
  return finish(c, "dk_stress");
}

dk_status dk_electrostatic_stress(dk_ctx* c, const double* rho, const double* vc, double* sigma) {
  if (!c) return DK_ERR_ARG;
  if (!rho || !vc || !sigma) return fail(c, DK_ERR_ARG, "dk_electrostatic_stress: null argument");
  if (c->n_local_atoms <= 0) return fail(c, DK_ERR_STATE, "dk_electrostatic_stress: dk_set_atoms has not been called");
  dk_status s = need_ws(c, electrostatic_stress_ws_bytes(c), "dk_electrostatic_stress");
  if (s != DK_OK) return s;
  hipSetDevice(c->device);
  {
    KTimer kt(c, DK_K_STRESS);
    DK_HIP(c, electrostatic_stress(c, rho, vc, sigma, c->ws));
  }
  return finish(c, "dk_electrostatic_stress");
}

dk_status dk_profile_enable(dk_ctx* c, int on) {
  if (!c) return DK_ERR_ARG;
  hipSetDevice(c->device);
  if (c->prof_on) prof_flush(c);
  if (on && c->prof_ev.empty()) {
    c->prof_ev.resize(4096);
    for (auto& e : c->prof_ev) DK_HIP(c, hipEventCreate(&e));
    c->prof_kind.assign(2048, 0);
  }
  c->prof_on = on != 0;
  c->prof_used = 0;
  for (int i = 0; i < DK_K_COUNT; ++i) { c->prof_ms[i] = 0; c->prof_cnt[i] = 0; }
  return DK_OK;
}

dk_status dk_profile_read(dk_ctx* c, double* ms, int64_t* counts) {
  if (!c || !ms || !counts) return DK_ERR_ARG;
  hipSetDevice(c->device);
  prof_flush(c);
  for (int i = 0; i < DK_K_COUNT; ++i) { ms[i] = c->prof_ms[i]; counts[i] = c->prof_cnt[i]; }
  return DK_OK;
}

dk_status dk_get_timings(const dk_ctx* c, double* ms, int n) {
  if (!c || !ms || n < 0) return DK_ERR_ARG;
  for (int i = 0; i < n && i < 8; ++i) ms[i] = c->timings[i];
  return DK_OK;
}

// ------------------------------------------------------ self-consistency --

dk_status dk_set_atoms(dk_ctx* c, int n_atoms, const double* pos, const dk_local_model* m) {
  if (!c) return DK_ERR_ARG;
  if (n_atoms <= 0 || !pos || !m) return fail(c, DK_ERR_ARG, "dk_set_atoms: need n_atoms > 0, positions and a model");
  if (!(m->rc > 0) || !(m->core_w2 > 0) || !std::isfinite(m->z) || !std::isfinite(m->core_amp))
    return fail(c, DK_ERR_ARG, "dk_set_atoms: model needs rc > 0, core_w2 > 0, finite z and core_amp");
  for (int i = 0; i < 3 * n_atoms; ++i)
    if (!std::isfinite(pos[i])) return fail(c, DK_ERR_NONFINITE, "dk_set_atoms: position %d not finite", i);
  hipSetDevice(c->device);
  free_atoms(c);
  DK_HIP(c, hipMalloc(&c->pos_dev, 3 * (size_t)n_atoms * sizeof(double)));
  DK_HIP(c, hipMalloc(&c->atom_tab, atom_tables_bytes(c, n_atoms)));
  DK_HIP(c, hipMalloc(&c->b_dev, c->ngrid * sizeof(double)));
  DK_HIP(c, hipMalloc(&c->vcore_dev, c->ngrid * sizeof(double)));
  DK_HIP(c, hipMemcpy(c->pos_dev, pos, 3 * (size_t)n_atoms * sizeof(double), hipMemcpyHostToDevice));
  c->n_local_atoms = n_atoms;
  c->loc_z = m->z;
  c->loc_rc = m->rc;
  c->loc_core_amp = m->core_amp;
  c->loc_core_w2 = m->core_w2;
  {
    KTimer kt(c, DK_K_SCF_FIELDS);
    DK_HIP(c, local_fields(c, c->pos_dev, n_atoms, m->z, m->rc, m->core_amp, m->core_w2,
                           c->atom_tab, c->b_dev, c->vcore_dev));
  }
  return finish(c, "dk_set_atoms");
}

dk_status dk_get_local_fields(dk_ctx* c, double* b, double* vcore) {
  if (!c) return DK_ERR_ARG;
  if (!c->n_local_atoms) return fail(c, DK_ERR_STATE, "dk_get_local_fields: no atoms set");
  hipSetDevice(c->device);
  if (b) DK_HIP(c, hipMemcpyAsync(b, c->b_dev, c->ngrid * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (vcore) DK_HIP(c, hipMemcpyAsync(vcore, c->vcore_dev, c->ngrid * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return finish(c, "dk_get_local_fields");
}

dk_status dk_start_density(dk_ctx* c, double* rho) {
  if (!c) return DK_ERR_ARG;
  if (!rho) return fail(c, DK_ERR_ARG, "dk_start_density: null pointer");
  if (!c->n_local_atoms) return fail(c, DK_ERR_STATE, "dk_start_density: no atoms set");
  hipSetDevice(c->device);
  {
    KTimer kt(c, DK_K_SCF_FIELDS);
    DK_HIP(c, negate(c, c->b_dev, rho));
  }
  return finish(c, "dk_start_density");
}

static dk_status run_poisson(dk_ctx* c, const double* src, double* v, double tol, int max_iter,
                             void* ws, int* iters, double* relres, const char* what) {
  int it = 0, st = 0;
  double rr = 0;
  {
    KTimer kt(c, DK_K_POISSON);
    DK_HIP(c, poisson_cg(c, src, v, tol, max_iter, ws, &it, &rr, &st));
  }
  if (iters) *iters = it;
  if (relres) *relres = rr;
  if (st == 2)
    return fail(c, DK_ERR_CONVERGENCE, "%s: %s reached %d iterations at relative residual %.3e",
                what, c->linear_solver == DK_SOLVER_AAR ? "AAR" : "CG", it, rr);
  return DK_OK;
}

dk_status dk_poisson(dk_ctx* c, const double* src, double* v, double tol, int max_iter, int* iters,
                     double* relres) {
  if (!c) return DK_ERR_ARG;
  if (!src || !v) return fail(c, DK_ERR_ARG, "dk_poisson: null pointer");
  if (!(tol > 0) || max_iter < 1) return fail(c, DK_ERR_ARG, "dk_poisson: need tol > 0, max_iter >= 1");
  dk_status s;
  if ((s = need_ws(c, ws_scf(c), "dk_poisson")) != DK_OK) return s;
  hipSetDevice(c->device);
  DK_HIP(c, check_finite(c, src, c->ngrid));
  if ((s = run_poisson(c, src, v, tol, max_iter, c->ws, iters, relres, "dk_poisson")) != DK_OK) return s;
  return finish(c, "dk_poisson");
}

dk_status dk_xc(dk_ctx* c, const double* rho, double* vxc, double* e_xc) {
  if (!c) return DK_ERR_ARG;
  if (!rho || !vxc) return fail(c, DK_ERR_ARG, "dk_xc: null pointer");
  dk_status s;
  if ((s = need_ws(c, ws_scf(c), "dk_xc")) != DK_OK) return s;
  hipSetDevice(c->device);
  double sums[4];
  {
    KTimer kt(c, DK_K_SCF_FIELDS);
    DK_HIP(c, effective_potential(c, rho, nullptr, nullptr, nullptr, vxc, nullptr, c->ws, sums));
  }
  if (e_xc) *e_xc = c->dv * sums[0];
  return finish(c, "dk_xc");
}

dk_status dk_scf_potential(dk_ctx* c, const double* rho, double* vc, double* veff, double tol,
                           int max_iter, dk_scf_terms* t) {
  if (!c) return DK_ERR_ARG;
  if (!rho || !vc || !veff || !t) return fail(c, DK_ERR_ARG, "dk_scf_potential: null pointer");
  if (!c->n_local_atoms) return fail(c, DK_ERR_STATE, "dk_scf_potential: no atoms set");
  if (!(tol > 0) || max_iter < 1) return fail(c, DK_ERR_ARG, "dk_scf_potential: need tol > 0, max_iter >= 1");
  dk_status s;
  if ((s = need_ws(c, ws_scf(c), "dk_scf_potential")) != DK_OK) return s;
  hipSetDevice(c->device);
  DK_HIP(c, check_finite(c, rho, c->ngrid));
  WsCursor cur(c->ws, ws_scf(c));
  void* pws = cur.take<char>(poisson_ws_bytes(c));
  double* src = cur.take<double>(c->ngrid);
  void* vws = cur.take<char>(potential_ws_bytes());
  if (!cur.ok) return fail(c, DK_ERR_ALLOC, "dk_scf_potential: workspace");
  {
    KTimer kt(c, DK_K_SCF_FIELDS);
    DK_HIP(c, add_fields(c, rho, c->b_dev, src));
  }
  int it = 0;
  double rr = 0;
  if ((s = run_poisson(c, src, vc, tol, max_iter, pws, &it, &rr, "dk_scf_potential")) != DK_OK) return s;
  double sums[4];
  {
    KTimer kt(c, DK_K_SCF_FIELDS);
    DK_HIP(c, effective_potential(c, rho, c->b_dev, vc, c->vcore_dev, nullptr, veff, vws, sums));
  }
  const double e_self = c->n_local_atoms * c->loc_z * c->loc_z / (std::sqrt(2.0 * M_PI) * c->loc_rc);
  t->e_xc = c->dv * sums[0];
  t->int_rho_vc = c->dv * sums[1];
  t->int_rho_vxc = c->dv * sums[2];
  t->e_es = 0.5 * c->dv * sums[3] - e_self;
  t->poisson_iters = it;
  t->poisson_relres = rr;
  t->reserved = 0;
  if ((s = finish(c, "dk_scf_potential")) != DK_OK) return s;
  return dk_set_potential(c, veff);
}

dk_status dk_pulay_bytes(const dk_ctx* c, int history, size_t* bytes) {
  if (!c || !bytes || history < 1 || history > kPulayMaxHistory) return DK_ERR_ARG;
  *bytes = pulay_state_bytes(c, history);
  return DK_OK;
}

dk_status dk_pulay_mix(dk_ctx* c, void* state, size_t state_bytes, int history, int iter,
                       double beta, const double* in, const double* out, double* next,
                       double* residual) {
  if (!c) return DK_ERR_ARG;
  if (!state || !in || !out || !next || !residual) return fail(c, DK_ERR_ARG, "dk_pulay_mix: null pointer");
  if (history < 1 || history > kPulayMaxHistory || iter < 0)
    return fail(c, DK_ERR_ARG, "dk_pulay_mix: need 1 <= history <= %d, iter >= 0", kPulayMaxHistory);
  if (next == in || next == out) return fail(c, DK_ERR_ARG, "dk_pulay_mix: next may not alias in or out");
  if (state_bytes < pulay_state_bytes(c, history))
    return fail(c, DK_ERR_ALLOC, "dk_pulay_mix: state of %zu bytes needed, %zu given", pulay_state_bytes(c, history), state_bytes);
  hipSetDevice(c->device);
  {
    KTimer kt(c, DK_K_MIX);
    DK_HIP(c, pulay_mix(c, state, history, iter, beta, in, out, next, residual));
  }
  if (!std::isfinite(*residual)) return fail(c, DK_ERR_NONFINITE, "dk_pulay_mix: non-finite residual");
  return finish(c, "dk_pulay_mix");
}

dk_status dk_kerker_pulay_bytes(const dk_ctx* c, int history, size_t* bytes) {
  if (!c || !bytes || history < 1 || history > kPulayMaxHistory) return DK_ERR_ARG;
  *bytes = kerker_pulay_state_bytes(c, history);
  return DK_OK;
}

dk_status dk_kerker_pulay_mix(dk_ctx* c, void* state, size_t state_bytes, int history, int iter,
                              int period, int restart, double beta, double k0, double tol,
                              const double* in, const double* out, double* next,
                              double* residual) {
  if (!c) return DK_ERR_ARG;
  if (!state || !in || !out || !next || !residual)
    return fail(c, DK_ERR_ARG, "dk_kerker_pulay_mix: null pointer");
  if (history < 1 || history > kPulayMaxHistory || iter < 0 || period < 1)
    return fail(c, DK_ERR_ARG, "dk_kerker_pulay_mix: need 1 <= history <= %d, iter >= 0, period >= 1",
                kPulayMaxHistory);
  if (!std::isfinite(beta) || !std::isfinite(k0) || !(tol > 0))
    return fail(c, DK_ERR_ARG, "dk_kerker_pulay_mix: beta, k0 must be finite and tol > 0");
  if (next == in || next == out) return fail(c, DK_ERR_ARG, "dk_kerker_pulay_mix: next may not alias in or out");
  if (restart && period > history)
    return fail(c, DK_ERR_ARG, "dk_kerker_pulay_mix: restarts need period <= history (%d > %d)",
                period, history);
  if (state_bytes < kerker_pulay_state_bytes(c, history))
    return fail(c, DK_ERR_ALLOC, "dk_kerker_pulay_mix: state of %zu bytes needed, %zu given",
                kerker_pulay_state_bytes(c, history), state_bytes);
  hipSetDevice(c->device);
  int cg_iters = 0, cg_status = 0;
  {
    KTimer kt(c, DK_K_MIX);
    DK_HIP(c, kerker_pulay_mix(c, state, history, iter, period, restart ? 1 : 0, beta, k0, tol,
                               20000, in, out, next, residual, &cg_iters, &cg_status));
  }
  if (cg_status == 2) return fail(c, DK_ERR_CONVERGENCE, "dk_kerker_pulay_mix: Kerker solve not converged");
  if (!std::isfinite(*residual)) return fail(c, DK_ERR_NONFINITE, "dk_kerker_pulay_mix: non-finite residual");
  return finish(c, "dk_kerker_pulay_mix");
}

dk_status dk_local_forces(dk_ctx* c, const double* rho, const double* vc, double* f) {
  if (!c) return DK_ERR_ARG;
  if (!rho || !vc || !f) return fail(c, DK_ERR_ARG, "dk_local_forces: null pointer");
  if (!c->n_local_atoms) return fail(c, DK_ERR_STATE, "dk_local_forces: no atoms set");
  dk_status s;
  if ((s = need_ws(c, ws_scf(c), "dk_local_forces")) != DK_OK) return s;
  hipSetDevice(c->device);
  double* fd = reinterpret_cast<double*>(c->ws);
  {
    KTimer kt(c, DK_K_SCF_FIELDS);
    DK_HIP(c, local_forces(c, c->atom_tab, c->n_local_atoms, c->loc_z, c->loc_rc, c->loc_core_amp,
                           rho, vc, fd));
  }
  DK_HIP(c, hipMemcpyAsync(f, fd, 3 * (size_t)c->n_local_atoms * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return finish(c, "dk_local_forces");
}

// --------------------------------------------------------- learned start --

static bool shape_ok(const dk_mlp_shape* s) {
  return s && s->n_in >= 1 && s->n_in <= 64 && s->hidden >= 1 && s->hidden <= 64 &&
         s->n_hidden_layers >= 1 && s->n_hidden_layers <= 8;
}

static size_t mlp_ws_total(const dk_mlp_shape* s, int64_t n_points) {
  return std::max(mlp_ws_bytes(s->n_in, s->hidden, s->n_hidden_layers, (long)n_points),
                  mlp_density_ws_bytes(s->n_in, s->hidden, s->n_hidden_layers));
}

dk_status dk_mlp_param_count(const dk_mlp_shape* s, int64_t* count) {
  if (!shape_ok(s) || !count) return DK_ERR_ARG;
  *count = (int64_t)mlp_params(s->n_in, s->hidden, s->n_hidden_layers);
  return DK_OK;
}

dk_status dk_mlp_workspace_bytes(const dk_mlp_shape* s, int64_t n_points, size_t* bytes) {
  if (!shape_ok(s) || !bytes || n_points < 1) return DK_ERR_ARG;
  *bytes = mlp_ws_total(s, n_points);
  return DK_OK;
}

dk_status dk_descriptors(dk_ctx* c, int n_atoms, const double* pos, int n_w, const double* widths,
                         float* desc) {
  if (!c) return DK_ERR_ARG;
  if (n_atoms <= 0 || !pos || n_w <= 0 || n_w > 64 || !widths || !desc)
    return fail(c, DK_ERR_ARG, "dk_descriptors: bad argument");
  for (int k = 0; k < n_w; ++k)
    if (!(widths[k] > 0)) return fail(c, DK_ERR_ARG, "dk_descriptors: widths must be positive");
  hipSetDevice(c->device);
  const int nmax = std::max(c->nx, std::max(c->ny, c->nz));
  double *pd = nullptr, *wd = nullptr, *tab = nullptr;
  DK_HIP(c, hipMalloc(&pd, 3 * (size_t)n_atoms * sizeof(double)));
  DK_HIP(c, hipMalloc(&wd, (size_t)n_w * sizeof(double)));
  DK_HIP(c, hipMalloc(&tab, desc_tables_bytes(n_atoms, n_w, nmax)));
  hipError_t e = hipMemcpy(pd, pos, 3 * (size_t)n_atoms * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(wd, widths, (size_t)n_w * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    KTimer kt(c, DK_K_MIX);
    e = descriptors(c, pd, n_atoms, n_w, wd, tab, desc);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(pd);
  hipFree(wd);
  hipFree(tab);
  if (e != hipSuccess) return hip_fail(c, e, "dk_descriptors");
  return finish(c, "dk_descriptors");
}

dk_status dk_descriptor_stats(dk_ctx* c, const float* desc, int64_t n, int n_w, double* mean,
                              double* inv_std) {
  if (!c) return DK_ERR_ARG;
  if (!desc || !mean || !inv_std || n < 1 || n_w < 1 || n_w > 64)
    return fail(c, DK_ERR_ARG, "dk_descriptor_stats: bad argument");
  hipSetDevice(c->device);
  double* part = nullptr;
  DK_HIP(c, hipMalloc(&part, channel_stats_ws_bytes(n_w)));
  hipError_t e;
  {
    KTimer kt(c, DK_K_MIX);
    e = channel_stats(c, desc, (long)n, n_w, mean, inv_std, part);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  hipFree(part);
  if (e != hipSuccess) return hip_fail(c, e, "dk_descriptor_stats");
  return finish(c, "dk_descriptor_stats");
}

dk_status dk_mlp_gather(dk_ctx* c, const float* desc, const double* rho, int n_w, const int64_t* idx,
                        int64_t n_pts, const double* mean, const double* inv_std, double scale,
                        float* u, float* t) {
  if (!c) return DK_ERR_ARG;
  if (!desc || !mean || !inv_std || !u || n_pts < 1 || n_w < 1 || (rho && !t))
    return fail(c, DK_ERR_ARG, "dk_mlp_gather: bad argument");
  hipSetDevice(c->device);
  {
    KTimer kt(c, DK_K_MIX);
    DK_HIP(c, mlp_gather(c, desc, rho, idx, n_w, (long)n_pts, mean, inv_std, scale, u, t));
  }
  return finish(c, "dk_mlp_gather");
}

static dk_status mlp_common(dk_ctx* c, const dk_mlp_shape* s, int mode, const float* params,
                            const float* u, int64_t n_pts, void* ws, size_t ws_bytes,
                            const char* what) {
  if (!shape_ok(s)) return fail(c, DK_ERR_ARG, "%s: bad network shape", what);
  if (mode != DK_MLP_BF16 && mode != DK_MLP_F32) return fail(c, DK_ERR_ARG, "%s: bad mode", what);
  if (!params || !u || !ws || n_pts < 1) return fail(c, DK_ERR_ARG, "%s: bad argument", what);
  if (ws_bytes < mlp_ws_bytes(s->n_in, s->hidden, s->n_hidden_layers, (long)n_pts))
    return fail(c, DK_ERR_ALLOC, "%s: workspace of %zu bytes needed", what,
                mlp_ws_bytes(s->n_in, s->hidden, s->n_hidden_layers, (long)n_pts));
  return DK_OK;
}

dk_status dk_mlp_loss_grad(dk_ctx* c, const dk_mlp_shape* s, int mode, const float* params,
                           const float* u, const float* t, int64_t n_pts, float* grad,
                           double* loss, void* ws, size_t ws_bytes) {
  if (!c) return DK_ERR_ARG;
  dk_status st = mlp_common(c, s, mode, params, u, n_pts, ws, ws_bytes, "dk_mlp_loss_grad");
  if (st != DK_OK) return st;
  if (!t || !loss) return fail(c, DK_ERR_ARG, "dk_mlp_loss_grad: need targets and a loss output");
  hipSetDevice(c->device);
  double sum = 0.0;
  {
    KTimer kt(c, DK_K_MIX);
    DK_HIP(c, mlp_run(c, mode, s->n_in, s->hidden, s->n_hidden_layers, params, u, t, (long)n_pts,
                      grad, nullptr, ws, &sum));
  }
  *loss = sum / (double)n_pts;
  if (!std::isfinite(*loss)) return fail(c, DK_ERR_NONFINITE, "dk_mlp_loss_grad: non-finite loss");
  return finish(c, "dk_mlp_loss_grad");
}

dk_status dk_mlp_forward(dk_ctx* c, const dk_mlp_shape* s, int mode, const float* params,
                         const float* u, int64_t n_pts, double* y, void* ws, size_t ws_bytes) {
  if (!c) return DK_ERR_ARG;
  dk_status st = mlp_common(c, s, mode, params, u, n_pts, ws, ws_bytes, "dk_mlp_forward");
  if (st != DK_OK) return st;
  if (!y) return fail(c, DK_ERR_ARG, "dk_mlp_forward: null output");
  hipSetDevice(c->device);
  double sum = 0.0;
  {
    KTimer kt(c, DK_K_MIX);
    DK_HIP(c, mlp_run(c, mode, s->n_in, s->hidden, s->n_hidden_layers, params, u, nullptr,
                      (long)n_pts, nullptr, y, ws, &sum));
  }
  return finish(c, "dk_mlp_forward");
}

dk_status dk_adam_step(dk_ctx* c, int64_t n, float* th, float* m, float* v, const float* g, int t,
                       double lr, double b1, double b2, double eps) {
  if (!c) return DK_ERR_ARG;
  if (n < 1 || !th || !m || !v || !g || t < 1 || !(lr > 0) || !(b1 >= 0 && b1 < 1) ||
      !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(c, DK_ERR_ARG, "dk_adam_step: bad argument");
  hipSetDevice(c->device);
  {
    KTimer kt(c, DK_K_MIX);
    DK_HIP(c, adam_update(c, (long)n, th, m, v, g, t, lr, b1, b2, eps));
  }
  return finish(c, "dk_adam_step");
}

dk_status dk_mlp_density(dk_ctx* c, const dk_mlp_shape* s, int mode, const float* params,
                         const float* desc, const double* mean, const double* inv_std, double n_e,
                         double* rho, void* ws, size_t ws_bytes) {
  if (!c) return DK_ERR_ARG;
  if (!shape_ok(s) || (mode != DK_MLP_BF16 && mode != DK_MLP_F32))
    return fail(c, DK_ERR_ARG, "dk_mlp_density: bad shape or mode");
  if (!params || !desc || !mean || !inv_std || !rho || !ws || !(n_e > 0))
    return fail(c, DK_ERR_ARG, "dk_mlp_density: bad argument");
  if (ws_bytes < mlp_density_ws_bytes(s->n_in, s->hidden, s->n_hidden_layers))
    return fail(c, DK_ERR_ALLOC, "dk_mlp_density: workspace of %zu bytes needed",
                mlp_density_ws_bytes(s->n_in, s->hidden, s->n_hidden_layers));
  hipSetDevice(c->device);
  {
    KTimer kt(c, DK_K_MIX);
    DK_HIP(c, mlp_density(c, mode, s->n_in, s->hidden, s->n_hidden_layers, params, desc, mean,
                          inv_std, n_e, rho, ws));
  }
  return finish(c, "dk_mlp_density");
}

// ---------------------------------------------------- molecular dynamics --

dk_status dk_verlet_kick(dk_ctx* c, int n_atoms, double* v, const double* f, double half_dt,
                         double mass) {
  if (!c) return DK_ERR_ARG;
  if (n_atoms <= 0 || !v || !f || !(mass > 0) || !std::isfinite(half_dt))
    return fail(c, DK_ERR_ARG, "dk_verlet_kick: bad argument");
  hipSetDevice(c->device);
  DK_HIP(c, md_kick(c, v, f, half_dt / mass, 3 * n_atoms));
  return finish(c, "dk_verlet_kick");
}

dk_status dk_isokinetic_kick(dk_ctx* c, int n_atoms, double* v, const double* f, double tau,
                             double mass) {
  if (!c) return DK_ERR_ARG;
  if (n_atoms <= 0 || !v || !f || !(mass > 0) || !std::isfinite(tau))
    return fail(c, DK_ERR_ARG, "dk_isokinetic_kick: bad argument");
  hipSetDevice(c->device);
  DK_HIP(c, md_isokinetic_kick(c, v, f, 1.0 / mass, tau, 3 * n_atoms));
  return finish(c, "dk_isokinetic_kick");
}

dk_status dk_verlet_drift(dk_ctx* c, int n_atoms, double* x, const double* v, double dt) {
  if (!c) return DK_ERR_ARG;
  if (n_atoms <= 0 || !x || !v || !std::isfinite(dt)) return fail(c, DK_ERR_ARG, "dk_verlet_drift: bad argument");
  hipSetDevice(c->device);
  DK_HIP(c, md_drift(c, x, v, dt, 3 * n_atoms));
  return finish(c, "dk_verlet_drift");
}

dk_status dk_kinetic_energy(dk_ctx* c, int n_atoms, const double* v, double mass, double* e) {
  if (!c) return DK_ERR_ARG;
  if (n_atoms <= 0 || !v || !e || !(mass > 0)) return fail(c, DK_ERR_ARG, "dk_kinetic_energy: bad argument");
  hipSetDevice(c->device);
  double* out = nullptr;
  DK_HIP(c, hipMalloc(&out, sizeof(double)));
  hipError_t err = md_kinetic(c, v, 3 * n_atoms, mass, out);
  if (err == hipSuccess) err = hipMemcpyAsync(e, out, sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
  hipFree(out);
  if (err != hipSuccess) return hip_fail(c, err, "dk_kinetic_energy");
  return finish(c, "dk_kinetic_energy");
}

dk_status dk_set_linear_solver(dk_ctx* c, int solver, double omega, double beta, int history,
                               int period) {
  if (!c) return DK_ERR_ARG;
  if (solver != DK_SOLVER_CG && solver != DK_SOLVER_AAR)
    return fail(c, DK_ERR_ARG, "dk_set_linear_solver: unknown solver %d", solver);
  if (solver == DK_SOLVER_AAR) {
    if (!(omega > 0) || !(beta > 0) || history < 1 || history > kPulayMaxHistory || period < 1)
      return fail(c, DK_ERR_ARG,
                  "dk_set_linear_solver: AAR needs omega > 0, beta > 0, 1 <= history <= %d, "
                  "period >= 1", kPulayMaxHistory);
    c->aar_omega = omega;
    c->aar_beta = beta;
    c->aar_history = history;
    c->aar_period = period;
  }
  c->linear_solver = solver;
  c->last_error.clear();
  return DK_OK;
}

dk_status dk_free_energy(dk_ctx* c, const dk_scf_terms* t, double e_band, double e_ent,
                         double* free_energy, double* xc_stress) {
  if (!c) return DK_ERR_ARG;
  if (!t || !free_energy) return fail(c, DK_ERR_ARG, "dk_free_energy: null pointer");
  // Harris-Foulkes form with the input density: the band and entropy terms
  // count int rho_in V_eff once; remove the potential energy of rho_in and add
  // the exchange-correlation and electrostatic energies
  *free_energy = e_band + e_ent - t->int_rho_vc - t->int_rho_vxc + t->e_xc + t->e_es;
  if (xc_stress) {
    const double d = (t->e_xc - t->int_rho_vxc) / (c->lx * c->ly * c->lz);
    for (int i = 0; i < 9; ++i) xc_stress[i] = (i % 4 == 0) ? d : 0.0;
  }
  if (!std::isfinite(*free_energy))
    return fail(c, DK_ERR_NONFINITE, "dk_free_energy: non-finite free energy");
  c->last_error.clear();
  return DK_OK;
}

dk_status dk_time_correlation(dk_ctx* c, const double* series, int64_t n_steps, int n_comp,
                              int max_lag, double dt, double scale, double* corr,
                              double* integral) {
  if (!c) return DK_ERR_ARG;
  if (!series || !corr || n_comp <= 0 || n_steps <= 0)
    return fail(c, DK_ERR_ARG, "dk_time_correlation: bad argument");
  if (max_lag <= 0 || max_lag > n_steps)
    return fail(c, DK_ERR_ARG, "dk_time_correlation: need 0 < max_lag <= n_steps (%d, %lld)",
                max_lag, (long long)n_steps);
  if (integral && !(dt > 0)) return fail(c, DK_ERR_ARG, "dk_time_correlation: need dt > 0");
  hipSetDevice(c->device);
  {
    KTimer kt(c, DK_K_OTHER);
    DK_HIP(c, time_correlation(c, series, (long)n_steps, n_comp, max_lag, dt, scale, corr,
                               integral));
  }
  return finish(c, "dk_time_correlation");
}

dk_status dk_deviatoric_stress(dk_ctx* c, const double* sigma, const double* v, int n_atoms,
                               double mass, int64_t n_steps, double* s) {
  if (!c) return DK_ERR_ARG;
  if (!sigma || !s || n_steps <= 0) return fail(c, DK_ERR_ARG, "dk_deviatoric_stress: bad argument");
  if (v && (n_atoms <= 0 || !(mass > 0)))
    return fail(c, DK_ERR_ARG, "dk_deviatoric_stress: velocities need n_atoms > 0 and mass > 0");
  hipSetDevice(c->device);
  {
    KTimer kt(c, DK_K_OTHER);
    DK_HIP(c, deviatoric_stress(c, sigma, v, n_atoms, mass, (long)n_steps, s));
  }
  return finish(c, "dk_deviatoric_stress");
}

}  // extern "C"
