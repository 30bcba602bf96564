// C ABI of libdelimit: plan creation (float64 tables built on the host and
// uploaded once), argument validation before any launch, workspace
// chunking, and the launch sequence of each layer call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace dlm {
int lsc_weight_splits(int64_t V, int m, int target);
}

using namespace dlm;

namespace {

thread_local std::string g_err;

dlm_status fail(dlm_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

dlm_status ok() {
  g_err.clear();
  return DLM_OK;
}

}  // namespace

dlm_status dlm::report(dlm_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

namespace {

dlm_status launched(int rc) {
  if (rc == 0) return DLM_OK;
  if (rc == -3)  // every launcher's code for an operand layout it does not take
    return fail(DLM_EINVAL, "no kernel takes this operand layout (shape, row stride or alignment)");
  return fail(DLM_EDEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

bool have_device() {
  int n = 0;
  return hipGetDeviceCount(&n) == hipSuccess && n > 0;
}

bool upload(DevMat &d, const std::vector<double> &h, int rows, int cols, hipStream_t st, std::vector<float> &sf,
            std::vector<uint16_t> &sh) {
  const size_t n = size_t(rows) * cols;
  d.rows = rows;
  d.cols = cols;
  if (!d.f32 && hipMalloc(&d.f32, std::max<size_t>(n, 1) * sizeof(float)) != hipSuccess) return false;
  if (!d.bf16 && hipMalloc(&d.bf16, std::max<size_t>(n, 1) * sizeof(uint16_t)) != hipSuccess) return false;
  sf.resize(n);
  sh.resize(n);
  for (size_t i = 0; i < n; ++i) {
    sf[i] = float(h[i]);
    sh[i] = f64_to_bf16_rne(h[i]);
  }
  if (hipMemcpyAsync(d.f32, sf.data(), n * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess) return false;
  if (hipMemcpyAsync(d.bf16, sh.data(), n * sizeof(uint16_t), hipMemcpyHostToDevice, st) != hipSuccess) return false;
  return true;
}

void release(DevMat &d) {
  if (d.f32) (void)hipFree(d.f32);
  if (d.bf16) (void)hipFree(d.bf16);
  d.f32 = nullptr;
  d.bf16 = nullptr;
}

std::vector<double> transpose(const std::vector<double> &a, int rows, int cols) {
  std::vector<double> t(size_t(rows) * cols);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) t[size_t(c) * rows + r] = a[size_t(r) * cols + c];
  return t;
}

bool finite_all(const double *p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

// ----------------------------------------------------------------- plans
struct dlm_sh_plan {
  int L = 0, K = 0, S = 0;
  double lambda = 0, b0_max = 0, rel_tol = 0;
  int64_t n_total = 0, n_dw = 0;
  std::vector<std::vector<int64_t>> members;
  std::vector<double> shell_b;
  std::vector<int64_t> dirs, offs;
  std::vector<std::vector<double>> B, P;  // host float64, B_s [N_s][K], P_s [K][N_s]
  bool uniform = true;
  // Whether every shell's fit (B^T B + lambda L) is positive definite.  A
  // plan without one still evaluates the basis (SH2Signal and its adjoint);
  // its P tables are zeros and every call that would read them fails.
  bool fit_ok = true;
  int singular_shell = -1;
  // device, all shells back to back: P [S][K][N], Pt [S][N][K], B [S][N][K], Bt [S][K][N]
  DevMat dP, dPt, dB, dBt;
  // the same four tables in MFMA fragment order for the per-shell kernel
  // (shell_frag_tables), all shells back to back; per-shell offsets in elements
  float *fragF[4] = {nullptr, nullptr, nullptr, nullptr};
  uint16_t *fragH[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<int64_t> frag_offF[4], frag_offH[4];
  // Bt in the accumulator order of the fused loss head (shell_frag_halves_acc),
  // same offsets as frag_offH[3]
  uint16_t *fragHacc = nullptr;
  std::vector<float> stage_ff;
  std::vector<uint16_t> stage_fh, stage_hacc;
  int n_b0 = 0;
  int32_t *d_dwidx = nullptr;  // [n_dw] creation-table index of each shell-major volume
  int32_t *d_b0idx = nullptr;  // [n_b0] creation-table indices of the b=0 volumes
  std::vector<float> stage_f;
  std::vector<uint16_t> stage_h;
  hipEvent_t staged = nullptr;
};

struct dlm_lsc_plan {
  int64_t m = 0;
  int T = 0, L_in = 0, L_out = 0, K_in = 0, K_out = 0;
  std::vector<int> ks;
  double alpha = 0, lambda = 0;
  std::vector<double> g, points, Bnb, Pm;
  std::vector<double> Q, pm1;  // Q[t][k][j] = (P_m B_t)[k][j]; pm1 = P_m 1
  DevMat dBnb, dBnbT, dPm, dPmT, dQ, dpm1;
};

namespace {

dlm_status sh_build_tables(dlm_sh_plan *p, const double *bvecs) {
  p->B.assign(p->S, {});
  p->P.assign(p->S, {});
  for (int s = 0; s < p->S; ++s) {
    const int64_t n = p->dirs[s];
    std::vector<double> u(size_t(n) * 3);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t src = p->members[s][i];
      if (!unit_dir(bvecs + 3 * src, u.data() + 3 * i))
        return fail(DLM_EINVAL, "gradient %lld (b=%g) is zero or not finite", (long long)src, p->shell_b[s]);
    }
    p->B[s].resize(size_t(n) * p->K);
    p->P[s].resize(size_t(n) * p->K);
    sh_basis_unit(p->L, u.data(), n, p->B[s].data());
  }
  // SH2Signal needs only the basis (evaluation on any table, Sec. 2.2); the
  // fit exists only where the regularised normal matrix is positive definite
  // (e.g. not for fewer directions than coefficients at lambda = 0).
  p->fit_ok = true;
  p->singular_shell = -1;
  for (int s = 0; s < p->S; ++s)
    if (!fit_from_basis(p->L, p->B[s].data(), p->dirs[s], p->lambda, p->P[s].data())) {
      std::fill(p->P[s].begin(), p->P[s].end(), 0.0);
      if (p->fit_ok) p->singular_shell = s;
      p->fit_ok = false;
    }
  return DLM_OK;
}

dlm_status no_fit(const dlm_sh_plan *p) {
  const int s = p->singular_shell;
  return fail(DLM_ESINGULAR,
              "shell %d (b=%g): the normal matrix of %lld directions at order %d and lambda %g is singular; "
              "this plan evaluates the basis (SH2Signal) only",
              s, p->shell_b[s], (long long)p->dirs[s], p->L, p->lambda);
}

dlm_status sh_upload(dlm_sh_plan *p, hipStream_t st) {
  if (p->staged) (void)hipEventSynchronize(p->staged);  // staging buffers free again
  std::vector<double> P, Pt, B, Bt;
  for (int s = 0; s < p->S; ++s) {
    const int n = int(p->dirs[s]);
    P.insert(P.end(), p->P[s].begin(), p->P[s].end());
    auto pt = transpose(p->P[s], p->K, n);
    Pt.insert(Pt.end(), pt.begin(), pt.end());
    B.insert(B.end(), p->B[s].begin(), p->B[s].end());
    auto bt = transpose(p->B[s], n, p->K);
    Bt.insert(Bt.end(), bt.begin(), bt.end());
  }
  const int total = int(p->n_dw);
  // Each table goes through its own staging slice so earlier async copies
  // never see a buffer overwritten by a later one.
  DevMat *dst[4] = {&p->dP, &p->dPt, &p->dB, &p->dBt};
  const std::vector<double> *src[4] = {&P, &Pt, &B, &Bt};
  const size_t n = size_t(total) * p->K;
  p->stage_f.resize(4 * n);
  p->stage_h.resize(4 * n);
  for (int t = 0; t < 4; ++t) {
    DevMat &d = *dst[t];
    if (!d.f32 && hipMalloc(&d.f32, n * sizeof(float)) != hipSuccess) return fail(DLM_ENOMEM, "hipMalloc failed");
    if (!d.bf16 && hipMalloc(&d.bf16, n * sizeof(uint16_t)) != hipSuccess) return fail(DLM_ENOMEM, "hipMalloc failed");
    float *f = p->stage_f.data() + t * n;
    uint16_t *h = p->stage_h.data() + t * n;
    for (size_t i = 0; i < n; ++i) {
      f[i] = float((*src[t])[i]);
      h[i] = f64_to_bf16_rne((*src[t])[i]);
    }
    if (hipMemcpyAsync(d.f32, f, n * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d.bf16, h, n * sizeof(uint16_t), hipMemcpyHostToDevice, st) != hipSuccess)
      return fail(DLM_EDEVICE, "table upload failed: %s", hipGetErrorString(hipGetLastError()));
  }
  // fragment-order copies: table t of shell s is [ncol][nred] = the
  // per-shell slice of P, Pt, B, Bt
  {
    size_t nf = 0, nh = 0;
    for (int t = 0; t < 4; ++t)
      for (int s = 0; s < p->S; ++s) {
        const int N = int(p->dirs[s]), K = p->K;
        const int ncol = (t == 0 || t == 3) ? K : N, nred = (t == 0 || t == 3) ? N : K;
        nf += shell_frag_floats(ncol, nred);
        nh += shell_frag_halves(ncol, nred);
      }
    p->stage_ff.resize(nf);
    p->stage_fh.resize(nh);
    size_t of = 0, oh = 0;
    for (int t = 0; t < 4; ++t) {
      const size_t f0 = of, h0 = oh;
      p->frag_offF[t].assign(p->S, 0);
      p->frag_offH[t].assign(p->S, 0);
      int64_t toff = 0;  // offset of shell s in the back-to-back table
      for (int s = 0; s < p->S; ++s) {
        const int N = int(p->dirs[s]), K = p->K;
        const int ncol = (t == 0 || t == 3) ? K : N, nred = (t == 0 || t == 3) ? N : K;
        p->frag_offF[t][s] = int64_t(of - f0);
        p->frag_offH[t][s] = int64_t(oh - h0);
        shell_frag_tables(src[t]->data() + toff, ncol, nred, p->stage_ff.data() + of, p->stage_fh.data() + oh);
        of += shell_frag_floats(ncol, nred);
        oh += shell_frag_halves(ncol, nred);
        toff += int64_t(N) * K;
      }
      const size_t cf = of - f0, ch = oh - h0;
      if (!p->fragF[t] && hipMalloc(&p->fragF[t], cf * sizeof(float)) != hipSuccess)
        return fail(DLM_ENOMEM, "hipMalloc failed");
      if (!p->fragH[t] && hipMalloc(&p->fragH[t], ch * sizeof(uint16_t)) != hipSuccess)
        return fail(DLM_ENOMEM, "hipMalloc failed");
      if (hipMemcpyAsync(p->fragF[t], p->stage_ff.data() + f0, cf * sizeof(float), hipMemcpyHostToDevice, st) !=
              hipSuccess ||
          hipMemcpyAsync(p->fragH[t], p->stage_fh.data() + h0, ch * sizeof(uint16_t), hipMemcpyHostToDevice, st) !=
              hipSuccess)
        return fail(DLM_EDEVICE, "table upload failed: %s", hipGetErrorString(hipGetLastError()));
    }
    size_t na = 0;
    for (int s = 0; s < p->S; ++s) na += shell_frag_halves(p->K, int(p->dirs[s]));
    p->stage_hacc.resize(na);
    size_t oa = 0;
    int64_t toff = 0;
    for (int s = 0; s < p->S; ++s) {
      const int N = int(p->dirs[s]), K = p->K;
      shell_frag_halves_acc(Bt.data() + toff, K, N, p->stage_hacc.data() + oa);
      oa += shell_frag_halves(K, N);
      toff += int64_t(N) * K;
    }
    if (!p->fragHacc && hipMalloc(&p->fragHacc, na * sizeof(uint16_t)) != hipSuccess)
      return fail(DLM_ENOMEM, "hipMalloc failed");
    if (hipMemcpyAsync(p->fragHacc, p->stage_hacc.data(), na * sizeof(uint16_t), hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return fail(DLM_EDEVICE, "table upload failed: %s", hipGetErrorString(hipGetLastError()));
  }
  if (!p->staged && hipEventCreateWithFlags(&p->staged, hipEventDisableTiming) != hipSuccess)
    return fail(DLM_EDEVICE, "hipEventCreate failed");
  if (hipEventRecord(p->staged, st) != hipSuccess) return fail(DLM_EDEVICE, "hipEventRecord failed");
  return DLM_OK;
}

}  // namespace

extern "C" {

const char *dlm_status_str(dlm_status s) {
  switch (s) {
    case DLM_OK: return "ok";
    case DLM_EINVAL: return "invalid argument";
    case DLM_ESINGULAR: return "singular fit";
    case DLM_ENOMEM: return "out of memory";
    case DLM_EDEVICE: return "device error";
    case DLM_EWORKSPACE: return "workspace too small";
  }
  return "unknown status";
}

const char *dlm_last_error(void) { return g_err.c_str(); }

int dlm_version(void) { return 1; }

dlm_status dlm_sh_basis(int sh_order, const double *dirs, int64_t n, double *B) {
  if (!sh_order_ok(sh_order)) return fail(DLM_EINVAL, "sh_order %d must be even and in [0, %d]", sh_order, kMaxShOrder);
  if (n < 0 || (n > 0 && (!dirs || !B))) return fail(DLM_EINVAL, "null pointer or negative n");
  const int K = sh_num_coeffs(sh_order);
  for (int64_t i = 0; i < n; ++i) {
    double u[3];
    if (!unit_dir(dirs + 3 * i, u)) return fail(DLM_EINVAL, "direction %lld is zero or not finite", (long long)i);
    sh_row(sh_order, u, B + i * K);
  }
  return ok();
}

dlm_status dlm_sh_fit_matrix(int sh_order, const double *dirs, int64_t n, double lb_lambda, double *P) {
  if (!sh_order_ok(sh_order)) return fail(DLM_EINVAL, "sh_order %d must be even and in [0, %d]", sh_order, kMaxShOrder);
  if (n <= 0 || !dirs || !P) return fail(DLM_EINVAL, "null pointer or n <= 0");
  if (!(lb_lambda >= 0.0) || !std::isfinite(lb_lambda)) return fail(DLM_EINVAL, "lb_lambda must be finite and >= 0");
  const int K = sh_num_coeffs(sh_order);
  std::vector<double> B(size_t(n) * K);
  dlm_status s = dlm_sh_basis(sh_order, dirs, n, B.data());
  if (s != DLM_OK) return s;
  if (!fit_from_basis(sh_order, B.data(), n, lb_lambda, P))
    return fail(DLM_ESINGULAR, "normal matrix of %lld directions at order %d is singular", (long long)n, sh_order);
  return ok();
}

dlm_status dlm_lsc_kernel_points(const double *g, int64_t m, const int *kernel_sizes, int n_rings,
                                 double angular_distance, double *points) {
  if (m <= 0 || !g || !points || !kernel_sizes) return fail(DLM_EINVAL, "null pointer or m <= 0");
  if (n_rings < 1) return fail(DLM_EINVAL, "need at least one ring");
  int T = 1;
  for (int r = 0; r < n_rings; ++r) {
    if (kernel_sizes[r] < 1) return fail(DLM_EINVAL, "ring %d has %d points", r, kernel_sizes[r]);
    T += kernel_sizes[r];
  }
  if (T > kMaxTaps) return fail(DLM_EINVAL, "kernel has %d taps (max %d)", T, kMaxTaps);
  if (!(angular_distance > 0.0) || !(angular_distance < 3.14159265358979323846))
    return fail(DLM_EINVAL, "angular_distance must be in (0, pi) radians");
  std::vector<double> u(size_t(m) * 3);
  for (int64_t i = 0; i < m; ++i)
    if (!unit_dir(g + 3 * i, u.data() + 3 * i)) return fail(DLM_EINVAL, "direction %lld is zero or not finite", (long long)i);
  kernel_points_unit(u.data(), m, kernel_sizes, n_rings, angular_distance, points);
  return ok();
}

// ----------------------------------------------------------------- SH plan
dlm_status dlm_sh_plan_create(const double *bvecs, const double *bvals, int64_t n, int sh_order, double lb_lambda,
                              double b0_max, double shell_rel_tol, dlm_sh_plan **out) {
  if (!out) return fail(DLM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!bvecs || !bvals || n <= 0) return fail(DLM_EINVAL, "null table or n <= 0");
  if (!sh_order_ok(sh_order)) return fail(DLM_EINVAL, "sh_order %d must be even and in [0, %d]", sh_order, kMaxShOrder);
  if (!(lb_lambda >= 0.0) || !std::isfinite(lb_lambda)) return fail(DLM_EINVAL, "lb_lambda must be finite and >= 0");
  if (!std::isfinite(b0_max) || !(shell_rel_tol >= 0.0) || !(shell_rel_tol < 1.0))
    return fail(DLM_EINVAL, "b0_max must be finite and shell_rel_tol in [0, 1)");
  if (!finite_all(bvals, n)) return fail(DLM_EINVAL, "b-values must be finite");
  if (!have_device()) return fail(DLM_EDEVICE, "no HIP device is available");
  dlm_sh_plan *p = new (std::nothrow) dlm_sh_plan();
  if (!p) return fail(DLM_ENOMEM, "host allocation failed");
  p->L = sh_order;
  p->K = sh_num_coeffs(sh_order);
  p->lambda = lb_lambda;
  p->b0_max = b0_max;
  p->rel_tol = shell_rel_tol;
  p->n_total = n;
  group_shells(bvals, n, b0_max, shell_rel_tol, p->members, p->shell_b);
  p->S = int(p->members.size());
  if (p->S == 0) {
    delete p;
    return fail(DLM_EINVAL, "no diffusion-weighted volumes (all b < %g)", b0_max);
  }
  int64_t off = 0;
  for (int s = 0; s < p->S; ++s) {
    p->dirs.push_back(int64_t(p->members[s].size()));
    p->offs.push_back(off);
    off += p->dirs.back();
    if (p->dirs[s] != p->dirs[0]) p->uniform = false;
  }
  p->n_dw = off;
  {
    std::vector<int32_t> dw, b0;
    for (int sh = 0; sh < p->S; ++sh)
      for (int64_t i : p->members[sh]) dw.push_back(int32_t(i));
    for (int64_t i = 0; i < n; ++i)
      if (bvals[i] < b0_max) b0.push_back(int32_t(i));
    p->n_b0 = int(b0.size());
    if (n > int64_t(0x7fffffff) || hipMalloc(&p->d_dwidx, dw.size() * 4) != hipSuccess ||
        hipMemcpy(p->d_dwidx, dw.data(), dw.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        (p->n_b0 > 0 && (hipMalloc(&p->d_b0idx, b0.size() * 4) != hipSuccess ||
                         hipMemcpy(p->d_b0idx, b0.data(), b0.size() * 4, hipMemcpyHostToDevice) != hipSuccess))) {
      dlm_sh_plan_destroy(p);
      return fail(DLM_ENOMEM, "volume index upload failed");
    }
  }
  dlm_status s = sh_build_tables(p, bvecs);
  if (s == DLM_OK) s = sh_upload(p, nullptr);
  if (s == DLM_OK && hipStreamSynchronize(nullptr) != hipSuccess) s = fail(DLM_EDEVICE, "upload failed");
  if (s != DLM_OK) {
    dlm_sh_plan_destroy(p);
    return s;
  }
  *out = p;
  return ok();
}

dlm_status dlm_sh_plan_info(const dlm_sh_plan *p, int *n_shells, int *K, int64_t *n_dw) {
  if (!p) return fail(DLM_EINVAL, "plan is NULL");
  if (n_shells) *n_shells = p->S;
  if (K) *K = p->K;
  if (n_dw) *n_dw = p->n_dw;
  return ok();
}

dlm_status dlm_sh_plan_shell(const dlm_sh_plan *p, int shell, int64_t *n_dirs, double *b, int64_t *volume_index) {
  if (!p) return fail(DLM_EINVAL, "plan is NULL");
  if (shell < 0 || shell >= p->S) return fail(DLM_EINVAL, "shell %d out of range [0, %d)", shell, p->S);
  if (n_dirs) *n_dirs = p->dirs[shell];
  if (b) *b = p->shell_b[shell];
  if (volume_index) std::copy(p->members[shell].begin(), p->members[shell].end(), volume_index);
  return ok();
}

dlm_status dlm_sh_plan_matrices(const dlm_sh_plan *p, int shell, double *B, double *P) {
  if (!p) return fail(DLM_EINVAL, "plan is NULL");
  if (shell < 0 || shell >= p->S) return fail(DLM_EINVAL, "shell %d out of range [0, %d)", shell, p->S);
  if (B) std::copy(p->B[shell].begin(), p->B[shell].end(), B);
  if (P) {
    if (!p->fit_ok) return no_fit(p);
    std::copy(p->P[shell].begin(), p->P[shell].end(), P);
  }
  return ok();
}

dlm_status dlm_sh_plan_fit_status(const dlm_sh_plan *p) {
  if (!p) return fail(DLM_EINVAL, "plan is NULL");
  return p->fit_ok ? ok() : no_fit(p);
}

dlm_status dlm_sh_plan_update_gradients(dlm_sh_plan *p, const double *bvecs, void *stream) {
  if (!p || !bvecs) return fail(DLM_EINVAL, "plan or bvecs is NULL");
  auto saved_B = p->B;
  auto saved_P = p->P;
  const bool had_fit = p->fit_ok;
  const int saved_shell = p->singular_shell;
  dlm_status s = sh_build_tables(p, bvecs);
  if (s == DLM_OK && had_fit && !p->fit_ok) s = no_fit(p);  // a plan with a fit keeps one
  if (s != DLM_OK) {
    p->B = saved_B;
    p->P = saved_P;
    p->fit_ok = had_fit;
    p->singular_shell = saved_shell;
    return s;
  }
  s = sh_upload(p, (hipStream_t)stream);
  return s == DLM_OK ? ok() : s;
}

void dlm_sh_plan_destroy(dlm_sh_plan *p) {
  if (!p) return;
  if (p->staged) {
    (void)hipEventSynchronize(p->staged);
    (void)hipEventDestroy(p->staged);
  }
  release(p->dP);
  release(p->dPt);
  for (int t = 0; t < 4; ++t) {
    if (p->fragF[t]) (void)hipFree(p->fragF[t]);
    if (p->fragH[t]) (void)hipFree(p->fragH[t]);
  }
  if (p->fragHacc) (void)hipFree(p->fragHacc);
  release(p->dB);
  release(p->dBt);
  if (p->d_dwidx) (void)hipFree(p->d_dwidx);
  if (p->d_b0idx) (void)hipFree(p->d_b0idx);
  delete p;
}

namespace {

enum class ShOp { S2shFwd, S2shBwd, Sh2sFwd, Sh2sBwd };

dlm_status sh_apply(const dlm_sh_plan *p, const float *in, float *out, int64_t V, dlm_precision prec, void *stream,
                    ShOp op) {
  if (!p) return fail(DLM_EINVAL, "plan is NULL");
  if (V < 0) return fail(DLM_EINVAL, "V must be >= 0");
  if (prec != DLM_FP32 && prec != DLM_BF16) return fail(DLM_EINVAL, "unknown precision %d", int(prec));
  if ((op == ShOp::S2shFwd || op == ShOp::S2shBwd) && !p->fit_ok) return no_fit(p);
  if (V == 0) return ok();
  if (!in || !out) return fail(DLM_EINVAL, "null device pointer");
  const int K = p->K, S = p->S;
  const int64_t ndw = p->n_dw;
  // signal side: [V][ndw], coefficient side: [V][S][K]
  const bool to_coef = (op == ShOp::S2shFwd || op == ShOp::Sh2sBwd);
  const DevMat &tab = op == ShOp::S2shFwd ? p->dP : op == ShOp::S2shBwd ? p->dPt : op == ShOp::Sh2sFwd ? p->dB : p->dBt;
  static const char *const tags[] = {"signal2sh_fwd", "signal2sh_bwd", "sh2signal_fwd", "sh2signal_bwd"};
  static const KernelOp kops[] = {kOpS2shFwd, kOpS2shBwd, kOpSh2sFwd, kOpSh2sBwd};
  const int shells = p->uniform ? 1 : S;
  for (int s0 = 0; s0 < shells; ++s0) {
    const int64_t N = p->dirs[s0];
    TableGemm t;
    t.M = V;
    t.groups = p->uniform ? S : 1;
    const int64_t sig_off = p->uniform ? 0 : p->offs[s0];
    const int64_t coef_off = p->uniform ? 0 : int64_t(s0) * K;
    const int64_t tab_off = sig_off * K;  // tables are back to back: offs[s] * K
    if (to_coef) {
      t.A = in + sig_off;
      t.lda = ndw;
      t.a_gs = N;
      t.C = out + coef_off;
      t.ldc = int64_t(S) * K;
      t.c_gs = K;
      t.N = K;
      t.K = int(N);
    } else {
      t.A = in + coef_off;
      t.lda = int64_t(S) * K;
      t.a_gs = K;
      t.C = out + sig_off;
      t.ldc = ndw;
      t.c_gs = N;
      t.N = int(N);
      t.K = K;
    }
    t.Bf = tab.f32 + tab_off;
    t.Bh = tab.bf16 + tab_off;
    t.b_gs = N * K;
    t.op = kops[int(op)];
    const double ng = double(t.groups);
    TimedScope ts(tags[int(op)], stream, double(V) * ng * (double(N) + K) * 4.0, 2.0 * double(V) * ng * N * K);
    int rc = 0;
    // one wave per 16 voxels x shell (tables in fragment order) for the
    // contractions over the coefficients (K <= 64: Signal2SH adjoint,
    // SH2Signal), for FP32 Signal2SH on large batches in its table-resident
    // form, and for BF16 reductions over up to 96 directions (Signal2SH,
    // SH2Signal adjoint) on large batches; the rest keep the tiled core,
    // which measured faster for them
    bool shell = false;
    if (shell_gemm_ok(t.N, t.K)) {
      const int ti = int(op);
      ShellGemm g;
      g.A = t.A;
      g.lda = t.lda;
      g.a_gs = t.a_gs;
      g.C = t.C;
      g.ldc = t.ldc;
      g.c_gs = t.c_gs;
      g.frag_f = p->fragF[ti] + p->frag_offF[ti][s0];
      g.frag_h = p->fragH[ti] + p->frag_offH[ti][s0];
      g.frag_gs_f = int64_t(shell_frag_floats(t.N, t.K) * sizeof(float));
      g.frag_gs_h = int64_t(shell_frag_halves(t.N, t.K) * sizeof(uint16_t));
      g.ncol = t.N;
      g.nred = t.K;
      g.groups = t.groups;
      g.V = V;
      g.op = t.op;
      shell = t.K <= 64 || shell_s2sh_resident(g, prec) || shell_long_bf16(g, prec);
      if (shell) rc = launch_shell_gemm(g, prec, stream);
    }
    if (!shell) rc = launch_table_gemm(t, prec, stream);
    if (rc != 0) return launched(rc);
  }
  return ok();
}

}  // namespace

size_t dlm_signal2sh_raw_workspace_bytes(int64_t V) { return align256(size_t(std::max<int64_t>(V, 1)) * 4); }

dlm_status dlm_signal2sh_fwd_raw(const dlm_sh_plan *p, const float *raw, float *c, int64_t V, void *ws,
                                 size_t ws_bytes, dlm_precision prec, void *stream) {
  if (!p) return fail(DLM_EINVAL, "plan is NULL");
  if (V < 0) return fail(DLM_EINVAL, "V must be >= 0");
  if (prec != DLM_FP32 && prec != DLM_BF16) return fail(DLM_EINVAL, "unknown precision %d", int(prec));
  if (p->n_b0 == 0) return fail(DLM_EINVAL, "the gradient table has no b=0 volume to normalise by");
  if (!p->fit_ok) return no_fit(p);
  if (V == 0) return ok();
  if (!raw || !c || !ws) return fail(DLM_EINVAL, "null device pointer");
  if (ws_bytes < dlm_signal2sh_raw_workspace_bytes(V)) return fail(DLM_EWORKSPACE, "workspace too small");
  float *inv = static_cast<float *>(ws);
  const int K = p->K, S = p->S;
  {
    TimedScope ts("b0_inverse_mean", stream, double(V) * (p->n_b0 + 1) * 4.0, double(V) * p->n_b0);
    if (launch_b0_inverse_mean(raw, p->n_total, p->d_b0idx, p->n_b0, V, inv, stream) != 0)
      return fail(DLM_EDEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
  }
  const int shells = p->uniform ? 1 : S;
  for (int s0 = 0; s0 < shells; ++s0) {
    const int64_t N = p->dirs[s0];
    const int64_t off = p->uniform ? 0 : p->offs[s0];
    const int groups = p->uniform ? S : 1;
    TimedScope ts("signal2sh_fwd_raw", stream, double(V) * groups * (double(N) + K) * 4.0,
                  2.0 * double(V) * groups * N * K);
    if (launch_s2sh_raw(raw, p->n_total, p->d_dwidx + off, inv, p->dP.f32 + off * K, p->dP.bf16 + off * K,
                        c + (p->uniform ? 0 : int64_t(s0) * K), int64_t(S) * K, V, groups, int(N), K, prec,
                        stream) != 0)
      return fail(DLM_EDEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
  }
  return ok();
}

dlm_status dlm_signal2sh_fwd(const dlm_sh_plan *p, const float *x, float *c, int64_t V, dlm_precision prec, void *st) {
  return sh_apply(p, x, c, V, prec, st, ShOp::S2shFwd);
}
dlm_status dlm_signal2sh_bwd(const dlm_sh_plan *p, const float *dc, float *dx, int64_t V, dlm_precision prec, void *st) {
  return sh_apply(p, dc, dx, V, prec, st, ShOp::S2shBwd);
}
dlm_status dlm_sh2signal_fwd(const dlm_sh_plan *p, const float *c, float *x, int64_t V, dlm_precision prec, void *st) {
  return sh_apply(p, c, x, V, prec, st, ShOp::Sh2sFwd);
}
dlm_status dlm_sh2signal_bwd(const dlm_sh_plan *p, const float *dx, float *dc, int64_t V, dlm_precision prec, void *st) {
  return sh_apply(p, dx, dc, V, prec, st, ShOp::Sh2sBwd);
}

int dlm_sh2signal_mse_supported(const dlm_sh_plan *p) {
  if (!p) return 0;
  for (int s = 0; s < p->S; ++s)
    if (!sh2s_mse_ok(int(p->dirs[s]), p->K)) return 0;
  return 1;
}

namespace {
int64_t sh2s_mse_waves(const dlm_sh_plan *p, int64_t V) {
  return p->uniform ? sh2s_mse_partials(V, p->S) : sh2s_mse_partials(V, 1) * p->S;
}
}  // namespace

size_t dlm_sh2signal_mse_workspace_bytes(const dlm_sh_plan *p, int64_t V) {
  if (!p) return 0;
  return align256(size_t(sh2s_mse_waves(p, std::max<int64_t>(V, 1)) + kSumBlocks) * 4);
}

dlm_status dlm_sh2signal_mse_fwd_bwd(const dlm_sh_plan *p, const float *c, const float *target, int64_t V,
                                     float *loss, float *dc, float *xhat, void *ws, size_t ws_bytes,
                                     dlm_precision prec, void *stream) {
  if (!p) return fail(DLM_EINVAL, "plan is NULL");
  if (V <= 0) return fail(DLM_EINVAL, "V must be > 0");
  if (prec != DLM_FP32 && prec != DLM_BF16) return fail(DLM_EINVAL, "unknown precision %d", int(prec));
  if (!dlm_sh2signal_mse_supported(p))
    return fail(DLM_EINVAL, "fused loss head needs <= 96 directions per shell and K <= 64");
  if (!c || !target || !loss || !dc || !ws) return fail(DLM_EINVAL, "null device pointer");
  if (dc == c) return fail(DLM_EINVAL, "dc must not alias c");
  if (ws_bytes < dlm_sh2signal_mse_workspace_bytes(p, V)) return fail(DLM_EWORKSPACE, "workspace too small");
  const int K = p->K, S = p->S;
  const int64_t ndw = p->n_dw;
  const double numel = double(V) * double(ndw);
  float *partials = static_cast<float *>(ws);
  const int shells = p->uniform ? 1 : S;
  int64_t pw = 0;
  for (int s0 = 0; s0 < shells; ++s0) {
    const int N = int(p->dirs[s0]);
    Sh2sMse t;
    t.groups = p->uniform ? S : 1;
    const int64_t sig_off = p->uniform ? 0 : p->offs[s0];
    const int64_t coef_off = p->uniform ? 0 : int64_t(s0) * K;
    t.c = c + coef_off;
    t.dc = dc + coef_off;
    t.ldcoef = int64_t(S) * K;
    t.K = K;
    t.target = target + sig_off;
    t.xhat = xhat ? xhat + sig_off : nullptr;
    t.ldsig = ndw;
    t.N = N;
    // B is table 2 ([N][K]), B^T table 3 ([K][N])
    t.fragB_f = p->fragF[2] + p->frag_offF[2][s0];
    t.fragB_h = p->fragH[2] + p->frag_offH[2][s0];
    t.fragBt_f = p->fragF[3] + p->frag_offF[3][s0];
    t.fragBt_h = p->fragHacc + p->frag_offH[3][s0];
    t.gsB_f = int64_t(shell_frag_floats(N, K) * sizeof(float));
    t.gsB_h = int64_t(shell_frag_halves(N, K) * sizeof(uint16_t));
    t.gsBt_f = int64_t(shell_frag_floats(K, N) * sizeof(float));
    t.gsBt_h = int64_t(shell_frag_halves(K, N) * sizeof(uint16_t));
    t.V = V;
    t.scale = float(2.0 / numel);
    t.partials = partials + pw;
    pw += sh2s_mse_partials(V, t.groups);
    const double ng = double(t.groups);
    TimedScope ts("sh2signal_mse", stream, double(V) * ng * (2.0 * K + N * (xhat ? 2.0 : 1.0)) * 4.0,
                  4.0 * double(V) * ng * N * K);
    if (launch_sh2s_mse(t, prec, stream) != 0)
      return fail(DLM_EDEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
  }
  if (launch_sum_scaled(partials, pw, loss, float(1.0 / numel), partials + pw, stream) != 0)
    return fail(DLM_EDEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
  return ok();
}

// ----------------------------------------------------------------- LSC plan
dlm_status dlm_lsc_plan_create(const double *sampled_gradients, int64_t m, int sh_order_in, int sh_order_out,
                               const int *kernel_sizes, int n_rings, double angular_distance, double lb_lambda,
                               dlm_lsc_plan **out) {
  if (!out) return fail(DLM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!sh_order_ok(sh_order_in) || !sh_order_ok(sh_order_out))
    return fail(DLM_EINVAL, "sh orders (%d, %d) must be even and in [0, %d]", sh_order_in, sh_order_out, kMaxShOrder);
  if (!(lb_lambda >= 0.0) || !std::isfinite(lb_lambda)) return fail(DLM_EINVAL, "lb_lambda must be finite and >= 0");
  if (m > (int64_t(1) << 20)) return fail(DLM_EINVAL, "m = %lld sampled directions is too many", (long long)m);
  if (!have_device()) return fail(DLM_EDEVICE, "no HIP device is available");
  dlm_lsc_plan *p = new (std::nothrow) dlm_lsc_plan();
  if (!p) return fail(DLM_ENOMEM, "host allocation failed");
  p->m = m;
  p->L_in = sh_order_in;
  p->L_out = sh_order_out;
  p->K_in = sh_num_coeffs(sh_order_in);
  p->K_out = sh_num_coeffs(sh_order_out);
  p->alpha = angular_distance;
  p->lambda = lb_lambda;
  if (n_rings >= 1 && kernel_sizes) p->ks.assign(kernel_sizes, kernel_sizes + n_rings);
  p->T = 1;
  for (int k : p->ks) p->T += k;
  p->points.resize(size_t(std::max<int64_t>(m, 0)) * p->T * 3);
  dlm_status s = dlm_lsc_kernel_points(sampled_gradients, m, kernel_sizes, n_rings, angular_distance, p->points.data());
  if (s != DLM_OK) {
    delete p;
    return s;
  }
  p->g.resize(size_t(m) * 3);
  for (int64_t i = 0; i < m; ++i) unit_dir(sampled_gradients + 3 * i, p->g.data() + 3 * i);
  const int64_t P = m * p->T;
  p->Bnb.resize(size_t(P) * p->K_in);
  sh_basis_unit(p->L_in, p->points.data(), P, p->Bnb.data());
  std::vector<double> Bm(size_t(m) * p->K_out);
  sh_basis_unit(p->L_out, p->g.data(), m, Bm.data());
  p->Pm.resize(size_t(m) * p->K_out);
  if (!fit_from_basis(p->L_out, Bm.data(), m, lb_lambda, p->Pm.data())) {
    delete p;
    return fail(DLM_ESINGULAR, "refit: normal matrix of %lld directions at order %d is singular", (long long)m,
                sh_order_out);
  }
  // Folded-form tables: Q_t = P_m B_t (B_t = rows i*T+t of B_nb), pm1 = P_m 1.
  const int Ki = p->K_in, Ko = p->K_out, T = p->T;
  p->Q.assign(size_t(T) * Ko * Ki, 0.0);
  for (int t = 0; t < T; ++t)
    for (int k = 0; k < Ko; ++k) {
      double *q = p->Q.data() + (size_t(t) * Ko + k) * Ki;
      for (int64_t i = 0; i < m; ++i) {
        const double pk = p->Pm[size_t(k) * m + i];
        const double *b = p->Bnb.data() + (size_t(i) * T + t) * Ki;
        for (int j = 0; j < Ki; ++j) q[j] += pk * b[j];
      }
    }
  p->pm1.assign(Ko, 0.0);
  for (int k = 0; k < Ko; ++k)
    for (int64_t i = 0; i < m; ++i) p->pm1[k] += p->Pm[size_t(k) * m + i];
  std::vector<float> sf;
  std::vector<uint16_t> shh;
  bool good = upload(p->dQ, p->Q, T, Ko * Ki, nullptr, sf, shh) && hipStreamSynchronize(nullptr) == hipSuccess;
  good = good && upload(p->dpm1, p->pm1, 1, Ko, nullptr, sf, shh) && hipStreamSynchronize(nullptr) == hipSuccess;
  good = good && upload(p->dBnb, p->Bnb, int(P), p->K_in, nullptr, sf, shh) && hipStreamSynchronize(nullptr) == hipSuccess;
  good = good && upload(p->dBnbT, transpose(p->Bnb, int(P), p->K_in), p->K_in, int(P), nullptr, sf, shh) &&
         hipStreamSynchronize(nullptr) == hipSuccess;
  good = good && upload(p->dPm, p->Pm, p->K_out, int(m), nullptr, sf, shh) && hipStreamSynchronize(nullptr) == hipSuccess;
  good = good && upload(p->dPmT, transpose(p->Pm, p->K_out, int(m)), int(m), p->K_out, nullptr, sf, shh) &&
         hipStreamSynchronize(nullptr) == hipSuccess;
  if (!good) {
    dlm_lsc_plan_destroy(p);
    return fail(DLM_EDEVICE, "table upload failed: %s", hipGetErrorString(hipGetLastError()));
  }
  *out = p;
  return ok();
}

dlm_status dlm_lsc_plan_info(const dlm_lsc_plan *p, int *T, int *K_in, int *K_out, int64_t *m) {
  if (!p) return fail(DLM_EINVAL, "plan is NULL");
  if (T) *T = p->T;
  if (K_in) *K_in = p->K_in;
  if (K_out) *K_out = p->K_out;
  if (m) *m = p->m;
  return ok();
}

dlm_status dlm_lsc_plan_tables(const dlm_lsc_plan *p, double *points, double *B_nb, double *P_m) {
  if (!p) return fail(DLM_EINVAL, "plan is NULL");
  if (points) std::copy(p->points.begin(), p->points.end(), points);
  if (B_nb) std::copy(p->Bnb.begin(), p->Bnb.end(), B_nb);
  if (P_m) std::copy(p->Pm.begin(), p->Pm.end(), P_m);
  return ok();
}

void dlm_lsc_plan_destroy(dlm_lsc_plan *p) {
  if (!p) return;
  release(p->dBnb);
  release(p->dBnbT);
  release(p->dPm);
  release(p->dPmT);
  release(p->dQ);
  release(p->dpm1);
  delete p;
}

namespace {

constexpr int kWeightSplitTarget = 256;
constexpr int64_t kMinChunk = 64;

struct LscWs {
  float *Wt = nullptr;
  uint16_t *Wh = nullptr, *Wth = nullptr;
  float *X = nullptr, *y = nullptr, *part = nullptr;
};

size_t lsc_ws_need(const dlm_lsc_plan *p, int C, int O, int64_t Vc) {
  const size_t CTO = size_t(C) * p->T * O;
  const size_t P = size_t(p->m) * p->T;
  size_t b = align256(CTO * 4) + 2 * align256(CTO * 2);
  b += align256(size_t(Vc) * C * P * 4);
  b += align256(size_t(Vc) * O * p->m * 4);
  b += align256(size_t(kWeightSplitTarget) * (size_t(C) * p->T + 1) * O * 4);
  return b;
}

LscWs lsc_ws_carve(const dlm_lsc_plan *p, int C, int O, int64_t Vc, void *ws) {
  LscWs w;
  char *b = static_cast<char *>(ws);
  const size_t CTO = size_t(C) * p->T * O;
  const size_t P = size_t(p->m) * p->T;
  w.Wt = reinterpret_cast<float *>(b);
  b += align256(CTO * 4);
  w.Wh = reinterpret_cast<uint16_t *>(b);
  b += align256(CTO * 2);
  w.Wth = reinterpret_cast<uint16_t *>(b);
  b += align256(CTO * 2);
  w.X = reinterpret_cast<float *>(b);
  b += align256(size_t(Vc) * C * P * 4);
  w.y = reinterpret_cast<float *>(b);
  b += align256(size_t(Vc) * O * p->m * 4);
  w.part = reinterpret_cast<float *>(b);
  return w;
}

// Largest chunk (multiple of kMinChunk unless V is smaller) whose workspace fits.
int64_t lsc_chunk(const dlm_lsc_plan *p, int C, int O, int64_t V, size_t ws_bytes) {
  int64_t hi = std::max<int64_t>(V, 1);
  // keep (chunk * m) within int range for the reduction index
  hi = std::min<int64_t>(hi, (int64_t(1) << 30) / std::max<int64_t>(p->m, 1));
  if (lsc_ws_need(p, C, O, hi) <= ws_bytes) return hi;
  int64_t lo = std::min<int64_t>(V, kMinChunk);
  if (lsc_ws_need(p, C, O, lo) > ws_bytes) return 0;
  // binary search on multiples of kMinChunk
  int64_t a = 1, b = hi / kMinChunk;
  if (b < 1) return lo;
  while (a < b) {
    const int64_t mid = (a + b + 1) / 2;
    if (lsc_ws_need(p, C, O, mid * kMinChunk) <= ws_bytes) a = mid;
    else b = mid - 1;
  }
  return a * kMinChunk;
}

struct FoldWs {
  float *Tw = nullptr, *TwT = nullptr, *bvec = nullptr, *part = nullptr, *dTw = nullptr;
  uint16_t *Twh = nullptr, *TwTh = nullptr;
};

constexpr int kFoldSplitMax = 128;

// The folded matrices (float32 and bfloat16 copies) keep rows padded with
// zeros to a multiple of 32 entries: the streaming core copies whole
// 32-entry slices.  Tw / Twh: [M][pad32(CK)]; TwT / TwTh: [CK][pad32(M)].
size_t pad32(size_t n) { return (n + 31) / 32 * 32; }

size_t fold_ws_need(const dlm_lsc_plan *p, int C, int O) {
  const size_t M = size_t(O) * p->K_out, CK = size_t(C) * p->K_in, N1 = CK + 1;
  return align256(M * pad32(CK) * 4) + align256(CK * pad32(M) * 4) + align256(M * pad32(CK) * 2) +
         align256(CK * pad32(M) * 2) + align256(M * 4) + align256(size_t(kFoldSplitMax) * M * N1 * 4) +
         align256(M * N1 * 4);
}

FoldWs fold_ws_carve(const dlm_lsc_plan *p, int C, int O, void *ws) {
  const size_t M = size_t(O) * p->K_out, CK = size_t(C) * p->K_in, N1 = CK + 1;
  char *b = static_cast<char *>(ws);
  FoldWs w;
  w.Tw = reinterpret_cast<float *>(b);
  b += align256(M * pad32(CK) * 4);
  w.TwT = reinterpret_cast<float *>(b);
  b += align256(CK * pad32(M) * 4);
  w.Twh = reinterpret_cast<uint16_t *>(b);
  b += align256(M * pad32(CK) * 2);
  w.TwTh = reinterpret_cast<uint16_t *>(b);
  b += align256(CK * pad32(M) * 2);
  w.bvec = reinterpret_cast<float *>(b);
  b += align256(M * 4);
  w.part = reinterpret_cast<float *>(b);
  b += align256(size_t(kFoldSplitMax) * M * N1 * 4);
  w.dTw = reinterpret_cast<float *>(b);
  return w;
}

dlm_status lsc_check(const dlm_lsc_plan *p, int C, int O, int64_t V, dlm_precision prec) {
  if (!p) return fail(DLM_EINVAL, "plan is NULL");
  if (C < 1 || C > kMaxChannels || O < 1 || O > kMaxChannels)
    return fail(DLM_EINVAL, "channels C=%d O=%d must be in [1, %d]", C, O, kMaxChannels);
  if (V < 0) return fail(DLM_EINVAL, "V must be >= 0");
  if (prec != DLM_FP32 && prec != DLM_BF16) return fail(DLM_EINVAL, "unknown precision %d", int(prec));
  return DLM_OK;
}

}  // namespace

dlm_status dlm_lsc_workspace_bytes(const dlm_lsc_plan *p, int C, int O, int64_t V_chunk, dlm_lsc_form form,
                                   dlm_precision prec, size_t *bytes) {
  dlm_status s = lsc_check(p, C, O, V_chunk, prec);
  if (s != DLM_OK) return s;
  if (!bytes) return fail(DLM_EINVAL, "bytes is NULL");
  if (form == DLM_LSC_FOLDED) *bytes = fold_ws_need(p, C, O);
  else if (form == DLM_LSC_RESAMPLE) *bytes = lsc_ws_need(p, C, O, std::max<int64_t>(V_chunk, 1));
  else return fail(DLM_EINVAL, "unknown LSC form %d", int(form));
  return ok();
}

namespace {

// The folded matrix for one use: T (forward, `transposed` false) or T^T
// (input gradient), in the precision's storage only (float32 or bfloat16),
// with its row padding zeroed.
dlm_status fold_weights(const dlm_lsc_plan *p, int C, int O, const float *W, const float *bias, const FoldWs &w,
                        bool transposed, dlm_precision prec, void *stream) {
  const double KK = double(p->K_out) * p->K_in, M = double(O) * p->K_out, CK = double(C) * p->K_in;
  const bool bf = prec == DLM_BF16;
  {
    TimedScope ts("lsc_fold", stream, (double(O) * C * p->T + p->T * KK) * 4.0 + M * CK * (bf ? 2.0 : 4.0),
                  2.0 * O * C * KK * p->T);
    const size_t M_ = size_t(O) * p->K_out, CK_ = size_t(C) * p->K_in;
    const size_t esz = bf ? 2 : 4;
    void *table = transposed ? (bf ? (void *)w.TwTh : (void *)w.TwT) : (bf ? (void *)w.Twh : (void *)w.Tw);
    const size_t rows = transposed ? CK_ : M_, cols = transposed ? M_ : CK_;
    if (launch_zero_cols(table, int64_t(rows), int64_t(cols * esz), int64_t(pad32(cols) * esz), stream) != 0)
      return launched(-1);
    float *Tw = !transposed && !bf ? w.Tw : nullptr, *TwT = transposed && !bf ? w.TwT : nullptr;
    uint16_t *Twh = !transposed && bf ? w.Twh : nullptr, *TwTh = transposed && bf ? w.TwTh : nullptr;
    if (launch_lsc_fold(W, p->dQ.f32, C, O, p->T, p->K_in, p->K_out, Tw, TwT, Twh, TwTh, int64_t(pad32(CK_)),
                        int64_t(pad32(M_)), stream) != 0)
      return launched(-1);
  }
  return launched(launch_lsc_bias_vec(bias, p->dpm1.f32, O, p->K_out, w.bvec, stream));
}

dlm_status lsc_fwd_folded(const dlm_lsc_plan *p, const void *a_in, int C, const float *W, const float *bias, int O,
                          void *a_out, int64_t V, int fuse_relu, int io, uint16_t *relu_bits, void *ws, size_t ws_bytes,
                          dlm_precision prec, void *stream) {
  if (ws_bytes < fold_ws_need(p, C, O))
    return fail(DLM_EWORKSPACE, "workspace of %zu bytes is below the %zu-byte minimum", ws_bytes, fold_ws_need(p, C, O));
  FoldWs w = fold_ws_carve(p, C, O, ws);
  dlm_status s = fold_weights(p, C, O, W, bias, w, false, prec, stream);
  if (s != DLM_OK) return s;
  const int M = O * p->K_out, CK = C * p->K_in;
  TableGemm t;  // a_out[v][(o,k)] = sum_{(c,j)} Tw[(o,k)][(c,j)] a_in[v][(c,j)] + bias[o] (P_m 1)[k]
  if (io & DLM_IO_IN_BF16) t.Ah = static_cast<const uint16_t *>(a_in);
  else t.A = static_cast<const float *>(a_in);
  t.lda = CK;
  t.Bf = w.Tw;
  t.Bh = w.Twh;
  t.ldb_f = t.ldb_h = int64_t(pad32(size_t(CK)));
  if (io & DLM_IO_OUT_BF16) t.Ch = static_cast<uint16_t *>(a_out);
  else t.C = static_cast<float *>(a_out);
  t.ldc = M;
  t.bias_n = w.bvec;
  t.M = V;
  t.N = M;
  t.K = CK;
  t.relu = fuse_relu ? 1 : 0;
  t.op = kOpFoldFwd;
  t.relu_bits_out = fuse_relu ? relu_bits : nullptr;
  TimedScope ts("lsc_folded_fwd", stream,
                double(V) * (CK * ((io & DLM_IO_IN_BF16) ? 2.0 : 4.0) + double(M) * ((io & DLM_IO_OUT_BF16) ? 2.0 : 4.0) +
                             (t.relu_bits_out ? M / 8.0 : 0.0)),
                2.0 * double(V) * M * CK);
  return launched(launch_table_gemm(t, prec, stream));
}

dlm_status lsc_bwd_folded(const dlm_lsc_plan *p, const void *a_in, int C, const float *W, int O, const void *a_out,
                          const void *da_out, void *da_in, float *dW, float *dbias, int64_t V, int relu_flags, int io,
                          const uint16_t *relu_bits, void *ws, size_t ws_bytes, dlm_precision prec, void *stream) {
  if (ws_bytes < fold_ws_need(p, C, O))
    return fail(DLM_EWORKSPACE, "workspace of %zu bytes is below the %zu-byte minimum", ws_bytes, fold_ws_need(p, C, O));
  FoldWs w = fold_ws_carve(p, C, O, ws);
  const int M = O * p->K_out, CK = C * p->K_in, N1 = CK + 1;
  if (dW && V > int64_t(0x7fffffff)) return fail(DLM_EINVAL, "V = %lld exceeds the 2^31-1 voxels of one call", (long long)V);
  dlm_status s;
  const bool in_h = io & DLM_IO_IN_BF16, out_h = io & DLM_IO_OUT_BF16;
  // DLM_RELU_OUT with a bfloat16 a_out is rejected by the caller
  const float *mask = (relu_flags & DLM_RELU_OUT) ? static_cast<const float *>(a_out) : nullptr;
  if (da_in && V > 0) {
    if ((s = fold_weights(p, C, O, W, nullptr, w, true, prec, stream)) != DLM_OK) return s;
    TableGemm t;  // da_in[v][(c,j)] = sum_{(o,k)} Tw[(o,k)][(c,j)] (da_out * [a_out > 0])[v][(o,k)]
    if (out_h) t.Ah = static_cast<const uint16_t *>(da_out);
    else t.A = static_cast<const float *>(da_out);
    t.mask = mask;
    t.lda = M;
    t.Bf = w.TwT;
    t.Bh = w.TwTh;
    t.ldb_f = t.ldb_h = int64_t(pad32(size_t(M)));
    const bool bits = (relu_flags & DLM_RELU_IN) && relu_bits;  // mask from the forward's ReLU bits
    if (in_h) {
      t.Ch = static_cast<uint16_t *>(da_in);
      t.out_mask_h = (relu_flags & DLM_RELU_IN) && !bits ? static_cast<const uint16_t *>(a_in) : nullptr;
    } else {
      t.C = static_cast<float *>(da_in);
      t.out_mask = (relu_flags & DLM_RELU_IN) && !bits ? static_cast<const float *>(a_in) : nullptr;
    }
    t.relu_bits_in = bits ? relu_bits : nullptr;
    t.ldc = CK;
    t.M = V;
    t.N = CK;
    t.K = M;
    t.op = kOpFoldBwdData;
    const double ob = out_h ? 2.0 : 4.0, ib = in_h ? 2.0 : 4.0;  // bytes per element
    const bool omask = t.out_mask || t.out_mask_h;
    TimedScope ts("lsc_folded_bwd_data", stream,
                  double(V) * (double(M) * (mask ? 2.0 : 1.0) * ob + CK * (omask ? 2.0 : 1.0) * ib +
                               (t.relu_bits_in ? CK / 8.0 : 0.0)),
                  2.0 * double(V) * M * CK);
    if ((s = launched(launch_table_gemm(t, prec, stream))) != DLM_OK) return s;
  }
  if (dW) {
    int splits = 0;
    if (V > 0) {
      splits = fold_grad_splits(V, M, N1);
      if (splits > kFoldSplitMax) return fail(DLM_EINVAL, "internal: too many splits");
      TimedScope ts("lsc_folded_grad", stream,
                    double(V) * (double(M) * (mask ? 2.0 : 1.0) * (out_h ? 2.0 : 4.0) + CK * (in_h ? 2.0 : 4.0)),
                    2.0 * double(V) * M * N1);
      if (in_h || out_h) {
        const int ks = fold_grad_split_len(V, splits);
        s = launched(launch_stream_grad(out_h ? nullptr : static_cast<const float *>(da_out),
                                        out_h ? static_cast<const uint16_t *>(da_out) : nullptr,
                                        in_h ? nullptr : static_cast<const float *>(a_in),
                                        in_h ? static_cast<const uint16_t *>(a_in) : nullptr, V, M, CK, splits, ks,
                                        w.part, prec, stream));
      } else {
        s = launched(launch_lsc_fold_grad(static_cast<const float *>(da_out), mask, static_cast<const float *>(a_in), V,
                                          M, CK, splits, w.part, prec, stream));
      }
      if (s != DLM_OK) return s;
    }
    {
      TimedScope ts("lsc_fold_reduce", stream, double(M) * N1 * 4.0, double(splits) * M * N1);
      if ((s = launched(launch_sum_partials(w.part, splits, int64_t(M) * N1, w.dTw, stream))) != DLM_OK) return s;
    }
    TimedScope ts("lsc_unfold", stream, (double(M) * N1 + p->T * double(p->K_out) * p->K_in + double(O) * C * p->T) * 4.0,
                  2.0 * O * C * p->T * double(p->K_out) * p->K_in);
    if ((s = launched(launch_lsc_unfold(w.dTw, p->dQ.f32, p->dpm1.f32, C, O, p->T, p->K_in, p->K_out, dW, dbias,
                                        stream))) != DLM_OK)
      return s;
  }
  return DLM_OK;
}

}  // namespace

namespace {
bool aligned16p(const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; }

// bfloat16 activation storage: BF16 folded form, rows of a multiple of 8
// entries, 16-byte aligned tensors
dlm_status io_check(const dlm_lsc_plan *p, int C, int O, int io, dlm_lsc_form form, dlm_precision prec,
                    const void *in0, const void *in1, const void *out0, const void *out1) {
  if (io & ~(DLM_IO_IN_BF16 | DLM_IO_OUT_BF16)) return fail(DLM_EINVAL, "unknown io flags 0x%x", io);
  if (io == 0) return DLM_OK;
  if (prec != DLM_BF16 || form != DLM_LSC_FOLDED)
    return fail(DLM_EINVAL, "bfloat16 activations need DLM_BF16 and the folded form");
  if ((io & DLM_IO_IN_BF16) && ((C * p->K_in) % 8 != 0 || !aligned16p(in0) || !aligned16p(in1)))
    return fail(DLM_EINVAL, "bfloat16 inputs need C*K_in (%d) a multiple of 8 and 16-byte aligned tensors",
                C * p->K_in);
  if ((io & DLM_IO_OUT_BF16) && ((O * p->K_out) % 8 != 0 || !aligned16p(out0) || !aligned16p(out1)))
    return fail(DLM_EINVAL, "bfloat16 outputs need O*K_out (%d) a multiple of 8 and 16-byte aligned tensors",
                O * p->K_out);
  return DLM_OK;
}
}  // namespace

dlm_status dlm_lsc_fwd_io(const dlm_lsc_plan *p, const void *a_in, int C, const float *W, const float *bias, int O,
                          void *a_out, int64_t V, int fuse_relu, int io_flags, uint16_t *relu_bits, dlm_lsc_form form,
                          void *ws, size_t ws_bytes, dlm_precision prec, void *stream) {
  if (io_flags == 0 && !relu_bits)
    return dlm_lsc_fwd(p, static_cast<const float *>(a_in), C, W, bias, O, static_cast<float *>(a_out), V, fuse_relu,
                       form, ws, ws_bytes, prec, stream);
  dlm_status s = lsc_check(p, C, O, V, prec);
  if (s != DLM_OK) return s;
  if ((s = io_check(p, C, O, io_flags, form, prec, a_in, nullptr, a_out, nullptr)) != DLM_OK) return s;
  if (relu_bits && (form != DLM_LSC_FOLDED || !fuse_relu || (O * p->K_out) % 16 != 0))
    return fail(DLM_EINVAL, "ReLU bits need the folded form, fuse_relu and O*K_out (%d) a multiple of 16",
                O * p->K_out);
  if (V == 0) return ok();
  if (!a_in || !W || !a_out || !ws) return fail(DLM_EINVAL, "null device pointer");
  s = lsc_fwd_folded(p, a_in, C, W, bias, O, a_out, V, fuse_relu, io_flags, relu_bits, ws, ws_bytes, prec, stream);
  return s == DLM_OK ? ok() : s;
}

dlm_status dlm_lsc_bwd_io(const dlm_lsc_plan *p, const void *a_in, int C, const float *W, int O, const void *a_out,
                          const void *da_out, void *da_in, float *dW, float *dbias, int64_t V, int relu_flags,
                          int io_flags, const uint16_t *relu_bits, dlm_lsc_form form, void *ws, size_t ws_bytes,
                          dlm_precision prec, void *stream) {
  if (io_flags == 0 && !relu_bits)
    return dlm_lsc_bwd(p, static_cast<const float *>(a_in), C, W, O, static_cast<const float *>(a_out),
                       static_cast<const float *>(da_out), static_cast<float *>(da_in), dW, dbias, V, relu_flags, form,
                       ws, ws_bytes, prec, stream);
  dlm_status s = lsc_check(p, C, O, V, prec);
  if (s != DLM_OK) return s;
  if (relu_bits && (form != DLM_LSC_FOLDED || !(relu_flags & DLM_RELU_IN) || (C * p->K_in) % 16 != 0))
    return fail(DLM_EINVAL, "ReLU bits need the folded form, DLM_RELU_IN and C*K_in a multiple of 16");
  if ((s = io_check(p, C, O, io_flags, form, prec, a_in, da_in, a_out, da_out)) != DLM_OK) return s;
  if (!ws) return fail(DLM_EINVAL, "workspace is NULL");
  if (relu_flags & ~(DLM_RELU_OUT | DLM_RELU_IN)) return fail(DLM_EINVAL, "unknown relu flags 0x%x", relu_flags);
  if ((relu_flags & DLM_RELU_OUT) && io_flags)
    return fail(DLM_EINVAL, "DLM_RELU_OUT with bfloat16 activations: mask in the next layer (DLM_RELU_IN) instead");
  if ((relu_flags & DLM_RELU_OUT) && relu_bits)
    return fail(DLM_EINVAL, "DLM_RELU_OUT with ReLU bits: mask in the next layer (DLM_RELU_IN) instead");
  if (dbias && !dW) return fail(DLM_EINVAL, "dbias without dW is not supported");
  if (V > 0 && (!a_in || !W || !da_out)) return fail(DLM_EINVAL, "null device pointer");
  s = lsc_bwd_folded(p, a_in, C, W, O, a_out, da_out, da_in, dW, dbias, V, relu_flags, io_flags, relu_bits, ws,
                     ws_bytes, prec, stream);
  return s == DLM_OK ? ok() : s;
}

dlm_status dlm_lsc_fwd(const dlm_lsc_plan *p, const float *a_in, int C, const float *W, const float *bias, int O,
                       float *a_out, int64_t V, int fuse_relu, dlm_lsc_form form, void *ws, size_t ws_bytes,
                       dlm_precision prec, void *stream) {
  dlm_status s = lsc_check(p, C, O, V, prec);
  if (s != DLM_OK) return s;
  if (form != DLM_LSC_RESAMPLE && form != DLM_LSC_FOLDED) return fail(DLM_EINVAL, "unknown LSC form %d", int(form));
  if (V == 0) return ok();
  if (!a_in || !W || !a_out || !ws) return fail(DLM_EINVAL, "null device pointer");
  if (form == DLM_LSC_FOLDED) {
    s = lsc_fwd_folded(p, a_in, C, W, bias, O, a_out, V, fuse_relu, 0, nullptr, ws, ws_bytes, prec, stream);
    return s == DLM_OK ? ok() : s;
  }
  const int64_t Vc = lsc_chunk(p, C, O, V, ws_bytes);
  if (Vc == 0)
    return fail(DLM_EWORKSPACE, "workspace of %zu bytes is below the %zu-byte minimum", ws_bytes,
                lsc_ws_need(p, C, O, std::min<int64_t>(V, kMinChunk)));
  LscWs w = lsc_ws_carve(p, C, O, Vc, ws);
  const int T = p->T, m = int(p->m);
  const int64_t P = p->m * T;
  const double CTO = double(C) * T * O;
  {
    TimedScope ts("lsc_prepare_weights", stream, CTO * 12.0, 0.0);
    if ((s = launched(launch_prepare_weights(W, w.Wt, w.Wh, w.Wth, C, O, T, stream))) != DLM_OK) return s;
  }
  for (int64_t v0 = 0; v0 < V; v0 += Vc) {
    const int64_t nv = std::min(Vc, V - v0);
    const double dnv = double(nv);
    TableGemm rs;  // resampling: X[(v,c)][p] = sum_j B_nb[p][j] a[(v,c)][j]
    rs.A = a_in + v0 * C * p->K_in;
    rs.lda = p->K_in;
    rs.Bf = p->dBnb.f32;
    rs.Bh = p->dBnb.bf16;
    rs.C = w.X;
    rs.ldc = P;
    rs.M = nv * C;
    rs.N = int(P);
    rs.K = p->K_in;
    rs.op = kOpResample;
    {
      TimedScope ts("lsc_resample", stream, dnv * C * (p->K_in + double(P)) * 4.0, 2.0 * dnv * C * p->K_in * double(P));
      if ((s = launched(launch_table_gemm(rs, prec, stream))) != DLM_OK) return s;
    }
    {
      TimedScope ts("lsc_contract_fwd", stream, dnv * (C * double(P) + double(O) * m) * 4.0, 2.0 * dnv * m * CTO);
      if ((s = launched(launch_lsc_contract_fwd(w.X, W, w.Wh, bias, w.y, nv, C, O, m, T, prec, stream))) != DLM_OK)
        return s;
    }
    TableGemm rf;  // refit: a_out[(v,o)][k] = sum_i P_m[k][i] y[(v,o)][i]
    rf.A = w.y;
    rf.lda = m;
    rf.Bf = p->dPm.f32;
    rf.Bh = p->dPm.bf16;
    rf.C = a_out + v0 * O * p->K_out;
    rf.ldc = p->K_out;
    rf.M = nv * O;
    rf.N = p->K_out;
    rf.K = m;
    rf.relu = fuse_relu ? 1 : 0;
    rf.op = kOpRefit;
    TimedScope ts("lsc_refit", stream, dnv * O * (double(m) + p->K_out) * 4.0, 2.0 * dnv * O * m * p->K_out);
    if ((s = launched(launch_table_gemm(rf, prec, stream))) != DLM_OK) return s;
  }
  return ok();
}

dlm_status dlm_lsc_bwd(const dlm_lsc_plan *p, const float *a_in, int C, const float *W, int O, const float *a_out,
                       const float *da_out, float *da_in, float *dW, float *dbias, int64_t V, int relu_flags,
                       dlm_lsc_form form, void *ws, size_t ws_bytes, dlm_precision prec, void *stream) {
  dlm_status s = lsc_check(p, C, O, V, prec);
  if (s != DLM_OK) return s;
  if (form != DLM_LSC_RESAMPLE && form != DLM_LSC_FOLDED) return fail(DLM_EINVAL, "unknown LSC form %d", int(form));
  if (!ws) return fail(DLM_EINVAL, "workspace is NULL");
  if (relu_flags & ~(DLM_RELU_OUT | DLM_RELU_IN)) return fail(DLM_EINVAL, "unknown relu flags 0x%x", relu_flags);
  if ((relu_flags & DLM_RELU_OUT) && !a_out && V > 0)
    return fail(DLM_EINVAL, "DLM_RELU_OUT needs the forward output a_out");
  if (dbias && !dW) return fail(DLM_EINVAL, "dbias without dW is not supported");
  if (V > 0 && (!a_in || !W || !da_out)) return fail(DLM_EINVAL, "null device pointer");
  if (form == DLM_LSC_FOLDED) {
    if (V > 0 && !W) return fail(DLM_EINVAL, "null device pointer");
    s = lsc_bwd_folded(p, a_in, C, W, O, a_out, da_out, da_in, dW, dbias, V, relu_flags, 0, nullptr, ws, ws_bytes,
                       prec, stream);
    return s == DLM_OK ? ok() : s;
  }
  const int T = p->T, m = int(p->m);
  const int64_t P = p->m * T;
  if (V == 0) {
    if (dW || dbias) {
      LscWs w0 = lsc_ws_carve(p, C, O, 1, ws);
      if (ws_bytes < lsc_ws_need(p, C, O, 1)) return fail(DLM_EWORKSPACE, "workspace too small");
      if (dW && (s = launched(launch_reduce_weight_partials(w0.part, 0, dW, dbias, C, O, T, 0, stream))) != DLM_OK)
        return s;
      if (!dW && dbias) return fail(DLM_EINVAL, "dbias without dW is not supported");
    }
    return ok();
  }
  if (!a_in || !W || !da_out) return fail(DLM_EINVAL, "null device pointer");
  if (dbias && !dW) return fail(DLM_EINVAL, "dbias without dW is not supported");
  const int64_t Vc = lsc_chunk(p, C, O, V, ws_bytes);
  if (Vc == 0)
    return fail(DLM_EWORKSPACE, "workspace of %zu bytes is below the %zu-byte minimum", ws_bytes,
                lsc_ws_need(p, C, O, std::min<int64_t>(V, kMinChunk)));
  LscWs w = lsc_ws_carve(p, C, O, Vc, ws);
  const double CTO = double(C) * T * O;
  {
    TimedScope ts("lsc_prepare_weights", stream, CTO * 12.0, 0.0);
    if ((s = launched(launch_prepare_weights(W, w.Wt, w.Wh, w.Wth, C, O, T, stream))) != DLM_OK) return s;
  }
  for (int64_t v0 = 0; v0 < V; v0 += Vc) {
    const int64_t nv = std::min(Vc, V - v0);
    const double dnv = double(nv);
    TableGemm rb;  // dy[(v,o)][i] = sum_k P_m[k][i] (da * [a_out > 0])[(v,o)][k]
    rb.A = da_out + v0 * O * p->K_out;
    rb.mask = (relu_flags & DLM_RELU_OUT) ? a_out + v0 * O * p->K_out : nullptr;
    rb.lda = p->K_out;
    rb.Bf = p->dPmT.f32;
    rb.Bh = p->dPmT.bf16;
    rb.C = w.y;
    rb.ldc = m;
    rb.M = nv * O;
    rb.N = m;
    rb.K = p->K_out;
    rb.op = kOpRefitBwd;
    {
      TimedScope ts("lsc_refit_bwd", stream, dnv * O * (p->K_out * (rb.mask ? 2.0 : 1.0) + m) * 4.0,
                    2.0 * dnv * O * m * p->K_out);
      if ((s = launched(launch_table_gemm(rb, prec, stream))) != DLM_OK) return s;
    }
    if (dW) {
      TableGemm rs;  // recompute the neighbourhood matrices X
      rs.A = a_in + v0 * C * p->K_in;
      rs.lda = p->K_in;
      rs.Bf = p->dBnb.f32;
      rs.Bh = p->dBnb.bf16;
      rs.C = w.X;
      rs.ldc = P;
      rs.M = nv * C;
      rs.N = int(P);
      rs.K = p->K_in;
      rs.op = kOpResample;
      {
        TimedScope ts("lsc_resample", stream, dnv * C * (p->K_in + double(P)) * 4.0,
                      2.0 * dnv * C * p->K_in * double(P));
        if ((s = launched(launch_table_gemm(rs, prec, stream))) != DLM_OK) return s;
      }
      const int splits = lsc_weight_splits(nv, m, kWeightSplitTarget);
      {
        TimedScope ts("lsc_bwd_weight", stream, dnv * (C * double(P) + double(O) * m) * 4.0,
                      2.0 * dnv * m * O * (double(C) * T + 1.0));
        if ((s = launched(launch_lsc_contract_bwd_weight(w.X, w.y, w.part, nv, C, O, m, T, splits, prec, stream))) !=
            DLM_OK)
          return s;
      }
      TimedScope ts("lsc_reduce_weight", stream, (double(C) * T + 1.0) * O * 4.0, double(splits) * (C * T + 1.0) * O);
      if ((s = launched(launch_reduce_weight_partials(w.part, splits, dW, dbias, C, O, T, v0 > 0, stream))) != DLM_OK)
        return s;
    }
    if (da_in) {
      {
        TimedScope ts("lsc_bwd_data", stream, dnv * (double(O) * m + C * double(P)) * 4.0, 2.0 * dnv * m * CTO);
        if ((s = launched(launch_lsc_contract_bwd_data(w.y, w.Wt, w.Wth, w.X, nv, C, O, m, T, prec, stream))) !=
            DLM_OK)
          return s;
      }
      TableGemm ra;  // da[(v,c)][j] = sum_p B_nb[p][j] dX[(v,c)][p]
      ra.A = w.X;
      ra.lda = P;
      ra.Bf = p->dBnbT.f32;
      ra.Bh = p->dBnbT.bf16;
      ra.C = da_in + v0 * C * p->K_in;
      ra.out_mask = (relu_flags & DLM_RELU_IN) ? a_in + v0 * C * p->K_in : nullptr;
      ra.ldc = p->K_in;
      ra.M = nv * C;
      ra.N = p->K_in;
      ra.K = int(P);
      ra.op = kOpResampleBwd;
      TimedScope ts("lsc_resample_bwd", stream, dnv * C * (double(P) + p->K_in * (ra.out_mask ? 2.0 : 1.0)) * 4.0,
                    2.0 * dnv * C * double(P) * p->K_in);
      if ((s = launched(launch_table_gemm(ra, prec, stream))) != DLM_OK) return s;
    }
  }
  return ok();
}

// ----------------------------------------------------------------- training
size_t dlm_mse_workspace_bytes(int64_t n) { return align256(size_t(mse_blocks(std::max<int64_t>(n, 1))) * 4); }

dlm_status dlm_mse_fwd_bwd(const float *pred, const float *target, int64_t n, float *loss, float *dpred, void *ws,
                           size_t ws_bytes, void *stream) {
  if (n <= 0) return fail(DLM_EINVAL, "n must be > 0");
  if (!pred || !target || !loss || !ws) return fail(DLM_EINVAL, "null device pointer");
  if (ws_bytes < dlm_mse_workspace_bytes(n)) return fail(DLM_EWORKSPACE, "workspace too small");
  const int nb = mse_blocks(n);
  TimedScope ts("mse", stream, double(n) * (dpred ? 12.0 : 8.0), 3.0 * double(n));
  dlm_status s = launched(launch_mse(pred, target, n, loss, dpred, static_cast<float *>(ws), nb, stream));
  return s == DLM_OK ? ok() : s;
}

dlm_status dlm_relmse_fwd_bwd(const float *pred, const float *target, int64_t n, float eps, float *loss,
                              float *dpred, void *ws, size_t ws_bytes, void *stream) {
  if (n <= 0) return fail(DLM_EINVAL, "n must be > 0");
  if (!pred || !target || !loss || !ws) return fail(DLM_EINVAL, "null device pointer");
  if (!(eps >= 0.0f) || !std::isfinite(eps)) return fail(DLM_EINVAL, "eps must be finite and >= 0");
  if (ws_bytes < dlm_mse_workspace_bytes(n)) return fail(DLM_EWORKSPACE, "workspace too small");
  const int nb = mse_blocks(n);
  TimedScope ts("relmse", stream, double(n) * (dpred ? 12.0 : 8.0), 5.0 * double(n));
  dlm_status s = launched(launch_relmse(pred, target, n, eps, loss, dpred, static_cast<float *>(ws), nb, stream));
  return s == DLM_OK ? ok() : s;
}

dlm_status dlm_adam_step(float *w, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
                         float eps, int64_t step, void *stream) {
  if (n < 0) return fail(DLM_EINVAL, "n must be >= 0");
  if (n == 0) return ok();
  if (!w || !g || !m || !v) return fail(DLM_EINVAL, "null device pointer");
  if (step < 1) return fail(DLM_EINVAL, "step is 1-based");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f)) return fail(DLM_EINVAL, "betas must be in [0,1)");
  const float c1 = float(1.0 - std::pow(double(beta1), double(step)));
  const float c2 = float(1.0 - std::pow(double(beta2), double(step)));
  TimedScope ts("adam", stream, double(n) * 28.0, 10.0 * double(n));
  dlm_status s = launched(launch_adam(w, g, m, v, n, lr, beta1, beta2, eps, c1, c2, stream));
  return s == DLM_OK ? ok() : s;
}

}  // extern "C"
