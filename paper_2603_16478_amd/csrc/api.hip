// C ABI entry points (include/adjoint.h): scene lifetime, adjoint setup,
// Krylov solve, gradient contractions.  Host orchestration only; all
// arithmetic of the step runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "adjoint.h"
#include "host_scene.h"

namespace adj {

struct GmresState {
  int j, active, restart, pad;
  double tol, res, rnorm;
};

// kernels (defined in the .hip kernel files)
void launch_tet_blocks(hipStream_t, int, const int*, const double*, const double*, const double*,
                       const double*, double, const double*, double*, int*);
void launch_assemble(hipStream_t, int, const int*, const int*, const double*, const int*, const int*,
                     const double*, double*);
void launch_vjp_tets(hipStream_t, int, const int*, const double*, const double*, const double*,
                     const double*, const double*, const double*, double, const double*, const double*,
                     double*, double*, double*, unsigned*, double*);
void launch_contact_blocks(hipStream_t, int, const int*, const double*, const double*, const double*,
                           double, double, double, int, double*, double*, double*, double*, double*);
void launch_contact_fold(hipStream_t, int, const int*, const int*, const double*, double*);
void launch_capacitance(hipStream_t, int, int, const int*, const int*, const int*, int, const double*,
                        const double*, const double*, double, double, double*);
void launch_vjp_contacts(hipStream_t, int, const int*, const double*, const double*, const double*,
                         const double*, double, double*, double*, unsigned*, double*);
void launch_vjp_vectors(hipStream_t, int, const double*, const double*, const double*, double, double*,
                        double*, double*);
void launch_fill_zero(hipStream_t, size_t, double*);
void launch_delassus(hipStream_t, int, int, const int*, const long long*, const int*, const double*,
                     double*, double*, double*);
double* launch_gauss_jordan(hipStream_t, int, int, double*, double*, int*);
void launch_spmv_csr3(hipStream_t, int, const long long*, const int*, const double*, const double*,
                      long long, const double*, const GmresState*, double*);
void launch_spmv_tasks(hipStream_t, int, const int4*, const long long*, const int*, const double*,
                       const double*, long long, const double*, const GmresState*, double*);
void launch_wb_gather(hipStream_t, int, int, const int*, const int*, const int*, const double*,
                      const double*, const double*, const GmresState*, double*);
void launch_wb_correct(hipStream_t, int, int, const int*, const int*, const int*, const double*,
                       const double*, const double*, double, const double*, const GmresState*, double*);
void launch_bsr_spmv(hipStream_t, int, const int*, const int*, const double*, const double*, double*,
                     long long, const GmresState*);
int gm_blocks(long long);
void launch_gm_dots(hipStream_t, long long, const double*, long long, const double*, GmresState*,
                    double*, unsigned*, double*);
void launch_gm_update(hipStream_t, long long, double*, long long, double*, GmresState*, double*,
                      unsigned*, double*, double*, double*, double*, double*, int);
void launch_gm_finish(hipStream_t, long long, const GmresState*, const double*, const double*,
                      const double*, const double*, long long, double*, double*);
void launch_axpy(hipStream_t, long long, double, const double*, double*);
void launch_residual(hipStream_t, long long, const double*, double*, double*, double*, unsigned*,
                     GmresState*, double*, double*);

}  // namespace adj

using namespace adj;

static thread_local std::string g_err;

static adj_status fail(adj_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(e_ == hipErrorOutOfMemory ? ADJ_E_OOM : ADJ_E_DEVICE,           \
                  std::string(#expr) + ": " + hipGetErrorString(e_));             \
  } while (0)

namespace {

template <class T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void**)p, n * sizeof(T));
}

template <class T>
hipError_t upload(T** p, const std::vector<T>& v) {
  hipError_t e = dalloc(p, v.size());
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

}  // namespace

struct adj_scene {
  HostScene hs;
  int nv = 0, nt = 0, nnzb = 0, max_contacts = 0;
  long long n3 = 0;
  int restart = 0;
  // constant device data
  int *d_tets = nullptr, *d_rowptr = nullptr, *d_col = nullptr, *d_row_of_slot = nullptr,
      *d_diag_slot = nullptr, *d_slot_ptr = nullptr, *d_slot_code = nullptr;
  double *d_Bt = nullptr, *d_vol = nullptr, *d_lmu = nullptr, *d_llam = nullptr, *d_E = nullptr,
         *d_nu = nullptr, *d_mass = nullptr;
  long long *d_Sp = nullptr, *d_STp = nullptr;
  int *d_Sj = nullptr, *d_STj = nullptr;
  double *d_Sx = nullptr, *d_STx = nullptr;
  int *d_Stasks = nullptr, *d_STtasks = nullptr;
  int nS_tasks = 0, nST_tasks = 0;
  // per-step
  double *d_tetblk = nullptr, *d_val = nullptr;
  int* d_err = nullptr;
  double *d_Wt = nullptr, *d_Q = nullptr, *d_kh = nullptr, *d_Kc = nullptr, *d_kmu = nullptr;
  int *d_row_c = nullptr, *d_row_i = nullptr, *d_cmap = nullptr, *d_c_row0 = nullptr,
      *d_c_nrow = nullptr, *d_cv = nullptr, *d_cv_ptr = nullptr;
  // Delassus cache
  std::vector<int> cv_cached;
  bool delassus_valid = false;
  size_t cap_ncv = 0, cap_m = 0;
  double *d_Y = nullptr, *d_D = nullptr, *d_Z = nullptr, *d_C = nullptr, *d_P = nullptr,
         *d_colbuf = nullptr, *d_tvec = nullptr;
  // current step
  int nc = 0, ncv = 0, m = 0, mp = 0;
  double* d_X = nullptr;  // the buffer (d_C or d_colbuf) holding the capacitance inverse
  double mu = 0.0;
  const int* cur_vid = nullptr;
  const double* cur_frame = nullptr;
  const double* cur_q = nullptr;
  bool setup_done = false;
  int delassus_rebuilt = 0;
  // Krylov workspace
  double *d_Vt = nullptr, *d_scale = nullptr, *d_H = nullptr, *d_cs = nullptr, *d_sn = nullptr,
         *d_g = nullptr, *d_hbuf = nullptr, *d_coef = nullptr, *d_partial = nullptr;
  unsigned* d_counter = nullptr;
  GmresState* d_state = nullptr;
  GmresState* h_state = nullptr;  // pinned
  double *d_t1 = nullptr, *d_u = nullptr, *d_y = nullptr, *d_r = nullptr, *d_b = nullptr,
         *d_dz = nullptr, *d_xt = nullptr;
  // live kernel timing (adj_profile_begin / adj_profile_end)
  int prof_kernel = -1;
  std::vector<hipEvent_t> prof_ev;
  size_t prof_used = 0;
};

static const size_t kMaxProfiled = 65536;

// Bracket one launch of kernel class `id` with events when it is profiled.
struct ProfScope {
  adj_scene* s;
  hipStream_t st;
  bool on;
  ProfScope(adj_scene* s_, int id, hipStream_t st_) : s(s_), st(st_), on(false) {
    if (s->prof_kernel != id || s->prof_used >= kMaxProfiled) return;
    if (s->prof_ev.size() < 2 * (s->prof_used + 1)) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
      }
      s->prof_ev.push_back(a);
      s->prof_ev.push_back(b);
    }
    on = hipEventRecord(s->prof_ev[2 * s->prof_used], st) == hipSuccess;
  }
  ~ProfScope() {
    if (!on) return;
    if (hipEventRecord(s->prof_ev[2 * s->prof_used + 1], st) == hipSuccess) s->prof_used++;
  }
};

static void free_scene(adj_scene* s) {
  if (!s) return;
  void* ptrs[] = {s->d_tets,     s->d_rowptr, s->d_col,   s->d_row_of_slot, s->d_diag_slot,
                  s->d_slot_ptr, s->d_slot_code, s->d_Bt, s->d_vol,         s->d_lmu,
                  s->d_llam,     s->d_E,      s->d_nu,    s->d_mass,        s->d_Sp,
                  s->d_STp,      s->d_Sj,     s->d_STj,   s->d_Sx,          s->d_STx,
                  s->d_tetblk,   s->d_val,    s->d_err,   s->d_Wt,          s->d_Q,
                  s->d_kh,       s->d_Kc,     s->d_kmu,   s->d_row_c,       s->d_row_i,
                  s->d_cmap,     s->d_c_row0, s->d_c_nrow, s->d_cv,         s->d_cv_ptr,
                  s->d_Y,        s->d_D,      s->d_Z,     s->d_C,           s->d_P,
                  s->d_colbuf,   s->d_tvec,   s->d_Vt,    s->d_scale,       s->d_H,
                  s->d_cs,       s->d_sn,     s->d_g,     s->d_hbuf,        s->d_coef,
                  s->d_partial,  s->d_counter, s->d_state, s->d_t1,         s->d_u,
                  s->d_y,        s->d_r,      s->d_b,     s->d_dz,          s->d_xt,
                  s->d_Stasks,   s->d_STtasks};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (s->h_state) (void)hipHostFree(s->h_state);
  for (hipEvent_t e : s->prof_ev) (void)hipEventDestroy(e);
  delete s;
}

static const int kMaxRestart = 128;

extern "C" const char* adj_last_error(void) { return g_err.c_str(); }

extern "C" adj_status adj_scene_create(const adj_scene_desc* desc, int32_t max_contacts,
                                       adj_scene** out) {
  if (!out) return fail(ADJ_E_ARG, "out is null");
  *out = nullptr;
  if (max_contacts < 0) return fail(ADJ_E_ARG, "max_contacts < 0");
  adj_scene* s = new (std::nothrow) adj_scene();
  if (!s) return fail(ADJ_E_OOM, "host allocation failed");
  std::string err;
  adj_status st = build_host_scene(desc, s->hs, err);
  if (st != ADJ_OK) {
    delete s;
    return fail(st, err);
  }
  HostScene& h = s->hs;
  s->nv = h.nv;
  s->nt = h.nt;
  s->nnzb = (int)h.col.size();
  s->n3 = 3LL * h.nv;
  s->max_contacts = max_contacts;
  s->restart = 64;
#define UP(dst, src)                                   \
  do {                                                 \
    hipError_t e_ = upload(&dst, src);                 \
    if (e_ != hipSuccess) {                            \
      free_scene(s);                                   \
      return fail(ADJ_E_OOM, "device upload failed");  \
    }                                                  \
  } while (0)
  std::vector<long long> Sp(h.Sp.begin(), h.Sp.end()), STp(h.STp.begin(), h.STp.end());
  UP(s->d_tets, h.tets);
  UP(s->d_rowptr, h.rowptr);
  UP(s->d_col, h.col);
  UP(s->d_row_of_slot, h.row_of_slot);
  UP(s->d_diag_slot, h.diag_slot);
  UP(s->d_slot_ptr, h.slot_ptr);
  UP(s->d_slot_code, h.slot_code);
  UP(s->d_Bt, h.Bt);
  UP(s->d_vol, h.vol);
  UP(s->d_lmu, h.lmu);
  UP(s->d_llam, h.llam);
  UP(s->d_E, h.E);
  UP(s->d_nu, h.nu);
  UP(s->d_mass, h.mass);
  UP(s->d_Sp, Sp);
  UP(s->d_STp, STp);
  UP(s->d_Sj, h.Sj);
  UP(s->d_STj, h.STj);
  UP(s->d_Sx, h.Sx);
  UP(s->d_STx, h.STx);
  UP(s->d_Stasks, h.S_tasks);
  UP(s->d_STtasks, h.ST_tasks);
  s->nS_tasks = (int)(h.S_tasks.size() / 4);
  s->nST_tasks = (int)(h.ST_tasks.size() / 4);
#undef UP
  bool ok = true;
  const size_t mc = (size_t)std::max(1, max_contacts);
  const size_t R = kMaxRestart;
  const size_t nblk = (size_t)gm_blocks(s->n3) + 300;
  ok &= dalloc(&s->d_tetblk, 90 * (size_t)s->nt) == hipSuccess;
  ok &= dalloc(&s->d_val, 9 * (size_t)s->nnzb) == hipSuccess;
  ok &= dalloc(&s->d_err, 4) == hipSuccess;
  ok &= dalloc(&s->d_Wt, 9 * mc) == hipSuccess;
  ok &= dalloc(&s->d_Q, 9 * mc) == hipSuccess;
  ok &= dalloc(&s->d_kh, 4 * mc) == hipSuccess;
  ok &= dalloc(&s->d_Kc, 9 * mc) == hipSuccess;
  ok &= dalloc(&s->d_kmu, 3 * mc) == hipSuccess;
  ok &= dalloc(&s->d_row_c, 3 * mc) == hipSuccess;
  ok &= dalloc(&s->d_row_i, 3 * mc) == hipSuccess;
  ok &= dalloc(&s->d_cmap, mc) == hipSuccess;
  ok &= dalloc(&s->d_c_row0, mc) == hipSuccess;
  ok &= dalloc(&s->d_c_nrow, mc) == hipSuccess;
  ok &= dalloc(&s->d_cv, mc) == hipSuccess;
  ok &= dalloc(&s->d_cv_ptr, mc + 1) == hipSuccess;
  ok &= dalloc(&s->d_tvec, 3 * mc) == hipSuccess;
  ok &= dalloc(&s->d_P, 32 * 32) == hipSuccess;
  ok &= dalloc(&s->d_Vt, (R + 1) * (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_scale, R + 2) == hipSuccess;
  ok &= dalloc(&s->d_H, (R + 1) * R) == hipSuccess;
  ok &= dalloc(&s->d_cs, R + 1) == hipSuccess;
  ok &= dalloc(&s->d_sn, R + 1) == hipSuccess;
  ok &= dalloc(&s->d_g, R + 2) == hipSuccess;
  ok &= dalloc(&s->d_hbuf, 260) == hipSuccess;
  ok &= dalloc(&s->d_coef, 130) == hipSuccess;
  ok &= dalloc(&s->d_partial, nblk * 130) == hipSuccess;
  ok &= dalloc(&s->d_counter, 16) == hipSuccess;
  ok &= dalloc(&s->d_state, 1) == hipSuccess;
  ok &= dalloc(&s->d_t1, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_u, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_y, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_r, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_b, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_dz, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_xt, (size_t)s->n3) == hipSuccess;
  ok &= hipHostMalloc((void**)&s->h_state, sizeof(GmresState), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    free_scene(s);
    return fail(ADJ_E_OOM, "device workspace allocation failed");
  }
  if (hipMemset(s->d_counter, 0, 16 * sizeof(unsigned)) != hipSuccess ||
      hipMemset(s->d_err, 0, 4 * sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    free_scene(s);
    return fail(ADJ_E_DEVICE, "device initialisation failed");
  }
  *out = s;
  return ADJ_OK;
}

extern "C" adj_status adj_scene_destroy(adj_scene* scene) {
  if (!scene) return fail(ADJ_E_ARG, "scene is null");
  (void)hipDeviceSynchronize();
  free_scene(scene);
  return ADJ_OK;
}

extern "C" adj_status adj_scene_info(const adj_scene* s, int64_t* out) {
  if (!s || !out) return fail(ADJ_E_ARG, "null argument");
  out[0] = s->nv;
  out[1] = s->nt;
  out[2] = s->nnzb;
  out[3] = (int64_t)s->hs.Li.size();
  out[4] = (int64_t)s->hs.Sj.size();
  out[5] = s->max_contacts;
  return ADJ_OK;
}

static adj_status grow(double** p, size_t* cap, size_t need) {
  if (need <= *cap && *p) return ADJ_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  if (dalloc(p, need) != hipSuccess) {
    *cap = 0;
    return fail(ADJ_E_OOM, "device allocation failed");
  }
  *cap = need;
  return ADJ_OK;
}

extern "C" adj_status adjoint_setup(adj_scene* s, const adj_contact_state* cst, const double* q,
                                    const adj_solve_opts* opts, void* stream) {
  if (!s || !cst || !q) return fail(ADJ_E_ARG, "null argument");
  if (cst->n_contacts < 0 || cst->n_contacts > s->max_contacts)
    return fail(ADJ_E_SHAPE, "n_contacts exceeds the scene's max_contacts");
  if (cst->n_contacts > 0 && (!cst->vid || !cst->fric || !cst->frame || !cst->delta || !cst->lambda))
    return fail(ADJ_E_ARG, "contact arrays missing");
  if (!std::isfinite(cst->mu) || cst->mu < 0) return fail(ADJ_E_ARG, "mu must be finite and >= 0");
  hipStream_t st = (hipStream_t)stream;
  const int nc = cst->n_contacts;
  const double h2 = s->hs.h * s->hs.h;
  // contact bookkeeping on the host: unique contact vertices, row layout
  std::vector<int> vid(nc), fric(nc);
  if (nc) {
    HIPCHK(hipMemcpyAsync(vid.data(), cst->vid, nc * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(fric.data(), cst->fric, nc * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  std::vector<int> cv, cv_ptr, cmap(nc), row_c, row_i, c_row0(nc), c_nrow(nc);
  for (int c = 0; c < nc; ++c) {
    if (vid[c] < 0 || vid[c] >= s->nv) return fail(ADJ_E_ARG, "contact vertex out of range");
    if (c > 0 && vid[c] < vid[c - 1]) return fail(ADJ_E_ARG, "contacts must be sorted by vertex");
    if (c == 0 || vid[c] != vid[c - 1]) {
      cv.push_back(vid[c]);
      cv_ptr.push_back(c);
    }
    cmap[c] = (int)cv.size() - 1;
    c_row0[c] = (int)row_c.size();
    c_nrow[c] = fric[c] ? 3 : 1;
    for (int i = 0; i < c_nrow[c]; ++i) {
      row_c.push_back(c);
      row_i.push_back(i);
    }
  }
  cv_ptr.push_back(nc);
  const int ncv = (int)cv.size(), m = (int)row_c.size();
  s->nc = nc;
  s->ncv = ncv;
  s->m = m;
  s->mu = cst->mu;
  s->cur_vid = cst->vid;
  s->cur_frame = cst->frame;
  s->cur_q = q;
  if (nc) {
    HIPCHK(hipMemcpyAsync(s->d_cmap, cmap.data(), nc * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_c_row0, c_row0.data(), nc * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_c_nrow, c_nrow.data(), nc * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_row_c, row_c.data(), m * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_row_i, row_i.data(), m * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_cv, cv.data(), ncv * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_cv_ptr, cv_ptr.data(), (ncv + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  }
  // a1 + a2: per-tet Jacobians, gather assembly of Acal^T
  {
    ProfScope p(s, 5, st);
    launch_tet_blocks(st, s->nt, s->d_tets, s->d_Bt, s->d_vol, s->d_lmu, s->d_llam, h2, q, s->d_tetblk,
                      s->d_err);
  }
  {
    ProfScope p(s, 6, st);
    launch_assemble(st, s->nnzb, s->d_slot_ptr, s->d_slot_code, s->d_tetblk, s->d_row_of_slot, s->d_col,
                    s->d_mass, s->d_val);
  }
  // a3: contact blocks folded into the diagonal blocks of Acal^T
  launch_contact_blocks(st, nc, cst->fric, cst->frame, cst->delta, cst->lambda, cst->mu, s->hs.eps, h2, 1,
                        s->d_Wt, s->d_Q, s->d_kh, s->d_Kc, s->d_kmu);
  launch_contact_fold(st, nc, cst->vid, s->d_diag_slot, s->d_Wt, s->d_val);
  // a4: Delassus (cached per contact vertex set), capacitance, its inverse
  s->delassus_rebuilt = 0;
  if (nc) {
    const bool reuse = opts ? opts->reuse_delassus != 0 : true;
    if (!(reuse && s->delassus_valid && cv == s->cv_cached)) {
      adj_status a;
      size_t capY = s->cap_ncv ? (size_t)s->nv * s->cap_ncv : 0, capD = s->cap_ncv * s->cap_ncv,
             capZ = capY;
      if ((size_t)ncv > s->cap_ncv) {
        capY = capZ = capD = 0;
      }
      if ((a = grow(&s->d_Y, &capY, (size_t)s->nv * ncv)) != ADJ_OK) return a;
      if ((a = grow(&s->d_Z, &capZ, (size_t)s->nv * ncv)) != ADJ_OK) return a;
      if ((a = grow(&s->d_D, &capD, (size_t)ncv * ncv)) != ADJ_OK) return a;
      s->cap_ncv = std::max(s->cap_ncv, (size_t)ncv);
      launch_delassus(st, s->nv, ncv, s->d_cv, s->d_STp, s->d_STj, s->d_STx, s->d_Y, s->d_D, s->d_Z);
      s->cv_cached = cv;
      s->delassus_valid = true;
      s->delassus_rebuilt = 1;
    }
    const int mp = ((m + 31) / 32) * 32;
    s->mp = mp;
    size_t capC = s->cap_m * s->cap_m, capB = capC;
    if ((size_t)mp > s->cap_m) capC = capB = 0;
    adj_status a;
    if ((a = grow(&s->d_C, &capC, (size_t)mp * mp)) != ADJ_OK) return a;
    if ((a = grow(&s->d_colbuf, &capB, (size_t)mp * mp)) != ADJ_OK) return a;
    s->cap_m = std::max(s->cap_m, (size_t)mp);
    launch_capacitance(st, m, mp, s->d_row_c, s->d_row_i, s->d_cmap, ncv, s->d_D, s->d_Q, s->d_kh, cst->mu,
                       h2, s->d_C);
    {
      ProfScope p(s, 7, st);
      s->d_X = launch_gauss_jordan(st, m, mp, s->d_C, s->d_colbuf, s->d_err);
    }
  }
  HIPCHK(hipGetLastError());
  s->setup_done = true;
  return ADJ_OK;
}

extern "C" adj_status adj_check_status(adj_scene* s, void* stream) {
  if (!s) return fail(ADJ_E_ARG, "scene is null");
  hipStream_t st = (hipStream_t)stream;
  int err[4];
  HIPCHK(hipMemcpyAsync(err, s->d_err, sizeof(err), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (err[0] == 1) return fail(ADJ_E_INVERTED, "a tet has det F <= 0");
  if (err[0] == 2) return fail(ADJ_E_SINGULAR, "capacitance block pivot is zero or not finite");
  return ADJ_OK;
}

// P x -> out (x and out distinct from the scratch vectors t1, u, tvec)
static void apply_precond(adj_scene* s, hipStream_t st, const double* x, long long stride,
                          const double* scale, const GmresState* state, double* out) {
  const double h2 = s->hs.h * s->hs.h;
  {
    ProfScope p(s, 0, st);
    launch_spmv_tasks(st, s->nS_tasks, (const int4*)s->d_Stasks, s->d_Sp, s->d_Sj, s->d_Sx, x, stride, scale,
                      state, s->d_t1);
  }
  double* u = (s->nc == 0) ? out : s->d_u;
  {
    ProfScope p(s, 1, st);
    launch_spmv_tasks(st, s->nST_tasks, (const int4*)s->d_STtasks, s->d_STp, s->d_STj, s->d_STx, s->d_t1, 0,
                      nullptr, state, u);
  }
  if (s->nc == 0) return;
  {
    ProfScope p(s, 2, st);
    launch_wb_gather(st, s->m, s->mp, s->d_row_c, s->d_row_i, s->cur_vid, s->d_Q, s->d_X, s->d_u, state,
                     s->d_tvec);
  }
  {
    ProfScope p(s, 3, st);
    launch_wb_correct(st, s->nv, s->ncv, s->d_cv_ptr, s->d_c_row0, s->d_c_nrow, s->d_Q, s->d_tvec, s->d_Z,
                      h2, s->d_u, state, out);
  }
}

extern "C" adj_status adjoint_solve(adj_scene* s, const double* dL_dq, const double* dL_dv, double* z,
                                    const adj_solve_opts* opts, adj_solve_info* info, void* stream) {
  if (!s || !dL_dq || !dL_dv || !z || !opts) return fail(ADJ_E_ARG, "null argument");
  if (!s->setup_done) return fail(ADJ_E_ARG, "adjoint_setup has not run");
  if (!(opts->rtol > 0) || opts->maxit <= 0 || opts->restart < 1 || opts->restart > kMaxRestart)
    return fail(ADJ_E_ARG, "invalid solve options");
  if (opts->prec != ADJ_FP64) return fail(ADJ_E_NOTIMPL, "only ADJ_FP64 is implemented in this build");
  hipStream_t st = (hipStream_t)stream;
  const long long n3 = s->n3;
  const long long stride = n3;
  const int R = opts->restart;
  // b = dL_dq + dL_dv / h
  HIPCHK(hipMemcpyAsync(s->d_b, dL_dq, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  launch_axpy(st, n3, 1.0 / s->hs.h, dL_dv, s->d_b);
  launch_fill_zero(st, (size_t)n3, z);
  launch_fill_zero(st, (size_t)n3, s->d_r);
  GmresState init{};
  init.restart = R;
  init.tol = 0.0;
  HIPCHK(hipMemcpyAsync(s->d_state, &init, sizeof(GmresState), hipMemcpyHostToDevice, st));
  launch_residual(st, n3, s->d_b, s->d_r, s->d_Vt, s->d_partial, s->d_counter, s->d_state, s->d_scale,
                  s->d_g);
  HIPCHK(hipMemcpyAsync(s->h_state, s->d_state, sizeof(GmresState), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double bnorm = s->h_state->rnorm;
  const double tol = opts->rtol * bnorm;
  GmresState cur = *s->h_state;
  cur.tol = tol;
  cur.restart = R;
  cur.active = (bnorm > tol) ? 1 : 0;
  HIPCHK(hipMemcpyAsync(s->d_state, &cur, sizeof(GmresState), hipMemcpyHostToDevice, st));
  int total = 0;
  double relres = (bnorm > 0) ? cur.rnorm / bnorm : 0.0;
  bool converged = !(bnorm > tol);
  const int chunk = 8;
  while (!converged && total < opts->maxit) {
    // one restart cycle
    int done_in_cycle = 0;
    while (true) {
      for (int k = 0; k < chunk; ++k) {
        apply_precond(s, st, s->d_Vt, stride, s->d_scale, s->d_state, s->d_y);
        {
          ProfScope p(s, 4, st);
          launch_bsr_spmv(st, s->nv, s->d_rowptr, s->d_col, s->d_val, s->d_y, s->d_Vt, stride, s->d_state);
        }
        {
          ProfScope p(s, 8, st);
          launch_gm_dots(st, n3, s->d_Vt, stride, s->d_scale, s->d_state, s->d_partial, s->d_counter,
                         s->d_hbuf);
        }
        {
          ProfScope p(s, 9, st);
          launch_gm_update(st, n3, s->d_Vt, stride, s->d_scale, s->d_state, s->d_partial, s->d_counter + 1,
                           s->d_hbuf, s->d_H, s->d_cs, s->d_sn, s->d_g, 0);
        }
        launch_gm_update(st, n3, s->d_Vt, stride, s->d_scale, s->d_state, s->d_partial, s->d_counter + 2,
                         s->d_hbuf, s->d_H, s->d_cs, s->d_sn, s->d_g, 1);
      }
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(s->h_state, s->d_state, sizeof(GmresState), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      done_in_cycle = s->h_state->j;
      if (!s->h_state->active || total + done_in_cycle >= opts->maxit) break;
    }
    total += done_in_cycle;
    // z += P (V y)
    launch_gm_finish(st, n3, s->d_state, s->d_H, s->d_g, s->d_scale, s->d_Vt, stride, s->d_coef, s->d_xt);
    apply_precond(s, st, s->d_xt, 0, nullptr, nullptr, s->d_dz);
    launch_axpy(st, n3, 1.0, s->d_dz, z);
    // true residual; restarts the next cycle from it
    launch_bsr_spmv(st, s->nv, s->d_rowptr, s->d_col, s->d_val, z, s->d_r, 0, nullptr);
    launch_residual(st, n3, s->d_b, s->d_r, s->d_Vt, s->d_partial, s->d_counter + 3, s->d_state,
                    s->d_scale, s->d_g);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(s->h_state, s->d_state, sizeof(GmresState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    relres = (bnorm > 0) ? s->h_state->rnorm / bnorm : 0.0;
    if (!std::isfinite(relres)) return fail(ADJ_E_SINGULAR, "non-finite residual in the Krylov solve");
    converged = s->h_state->rnorm <= tol;
    if (done_in_cycle == 0 && !converged) break;  // no progress possible
  }
  if (info) {
    info->iters = total;
    info->refine_steps = 0;
    info->n_contacts = s->nc;
    info->m_rows = s->m;
    info->relres = relres;
    info->delassus_rebuilt = s->delassus_rebuilt;
  }
  if (!converged) return fail(ADJ_E_NOCONV, "Krylov solve did not reach rtol");
  return ADJ_OK;
}

extern "C" adj_status vjp_params(adj_scene* s, const double* z, const double* dL_dv, double* dL_dqbar,
                                 double* dL_dvbar, double* dL_dfext, double* grad3, double* dE_tet,
                                 double* dnu_tet, void* stream) {
  if (!s || !z || !dL_dv || !dL_dqbar || !dL_dvbar || !dL_dfext || !grad3)
    return fail(ADJ_E_ARG, "null argument");
  if (!s->setup_done) return fail(ADJ_E_ARG, "adjoint_setup has not run");
  hipStream_t st = (hipStream_t)stream;
  const double h = s->hs.h, h2 = h * h;
  launch_vjp_vectors(st, s->nv, z, dL_dv, s->d_mass, h, dL_dqbar, dL_dvbar, dL_dfext);
  launch_vjp_contacts(st, s->nc, s->cur_vid, s->cur_frame, s->d_Kc, s->d_kmu, z, h2, dL_dqbar,
                      s->d_partial, s->d_counter + 4, grad3);
  launch_vjp_tets(st, s->nt, s->d_tets, s->d_Bt, s->d_vol, s->d_lmu, s->d_llam, s->d_E, s->d_nu, h2,
                  s->cur_q, z, dE_tet, dnu_tet, s->d_partial + 4096, s->d_counter + 5, grad3);
  HIPCHK(hipGetLastError());
  return ADJ_OK;
}

extern "C" adj_status adj_profile_begin(adj_scene* s, int32_t kernel) {
  if (!s || kernel < 0 || kernel > 9) return fail(ADJ_E_ARG, "bad profile request");
  s->prof_kernel = kernel;
  s->prof_used = 0;
  return ADJ_OK;
}

extern "C" adj_status adj_profile_end(adj_scene* s, double* total_ms, int64_t* launches) {
  if (!s || !total_ms || !launches) return fail(ADJ_E_ARG, "null argument");
  double tot = 0.0;
  for (size_t i = 0; i < s->prof_used; ++i) {
    HIPCHK(hipEventSynchronize(s->prof_ev[2 * i + 1]));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, s->prof_ev[2 * i], s->prof_ev[2 * i + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)s->prof_used;
  s->prof_kernel = -1;
  s->prof_used = 0;
  return ADJ_OK;
}

extern "C" adj_status adj_debug_export(const adj_scene* s, int32_t what, void* host_out,
                                       int64_t capacity_bytes, int64_t* size_bytes) {
  if (!s || !size_bytes) return fail(ADJ_E_ARG, "null argument");
  const void* src = nullptr;
  int64_t bytes = 0;
  switch (what) {
    case 0: src = s->d_val; bytes = 9LL * s->nnzb * 8; break;
    case 1: src = s->d_rowptr; bytes = (s->nv + 1LL) * 4; break;
    case 2: src = s->d_col; bytes = (int64_t)s->nnzb * 4; break;
    case 3: src = s->d_X; bytes = (int64_t)s->mp * s->mp * 8; break;
    case 4: src = s->d_D; bytes = (int64_t)s->ncv * s->ncv * 8; break;
    case 5: src = s->d_Q; bytes = 9LL * s->nc * 8; break;
    default: return fail(ADJ_E_ARG, "unknown array");
  }
  *size_bytes = bytes;
  if (!host_out || capacity_bytes < bytes) return fail(ADJ_E_SHAPE, "buffer too small");
  HIPCHK(hipDeviceSynchronize());
  if (bytes) HIPCHK(hipMemcpy(host_out, src, bytes, hipMemcpyDeviceToHost));
  return ADJ_OK;
}

extern "C" adj_status sim_forward_step(adj_scene* s, const double* qbar, const double* vbar,
                                       const double* f_ext, double mu, double* q, double* v,
                                       adj_contact_state* contacts, void* stream) {
  (void)s; (void)qbar; (void)vbar; (void)f_ext; (void)mu; (void)q; (void)v; (void)contacts;
  (void)stream;
  return fail(ADJ_E_NOTIMPL, "sim_forward_step is not implemented in this build");
}
