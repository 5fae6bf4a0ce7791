// C ABI entry points (include/adjoint.h): scene lifetime, adjoint setup,
// Krylov solve, gradient contractions.  Host orchestration only; all
// arithmetic of the step runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "adjoint.h"
#include "host_scene.h"
#include "krylov_state.h"

namespace adj {


// kernels (defined in the .hip kernel files)
void launch_tet_blocks(hipStream_t, int, const int*, const double*, const double*, const double*,
                       const double*, double, const double*, double*, int*, int);
void launch_assemble(hipStream_t, int, int, const int*, const int*, const double*, const int*, const int*,
                     const double*, double*);
void launch_vjp_tets(hipStream_t, int, const int*, const double*, const double*, const double*,
                     const double*, const double*, const double*, double, const double*, const double*,
                     double*, double*, double*, double*, int);
void launch_contact_blocks(hipStream_t, int, const int*, const double*, const double*, const double*,
                           double, const double*, double, double, int, double*, double*, double*, double*,
                           double*);
void launch_contact_fold(hipStream_t, int, const int*, const int*, const double*, double*);
void launch_binding_fold(hipStream_t, int, const int*, const double*, double, const int*, double*);
void launch_binding_force(hipStream_t, int, const int*, const double*, double, const double*, const double*,
                          double*);
void launch_binding_vjp(hipStream_t, int, const int*, const double*, double, const double*, const double*,
                        const double*, double*, double*);
void launch_capacitance(hipStream_t, int, int, const int*, const int*, const int*, int, const double*,
                        const double*, const double*, double, double, int, double*);
void launch_vjp_contacts(hipStream_t, int, const int*, const double*, const double*, const double*,
                         const double*, double, double*, double*, double*, double*);
void launch_vjp_vectors(hipStream_t, int, const double*, const double*, const double*, double, double*,
                        double*, double*);
void launch_fill_zero(hipStream_t, size_t, double*);
void launch_fill_int(hipStream_t, size_t, int*, int);
void launch_actuation_force(hipStream_t, int, int, const int*, const double*, const double*, const double*,
                            const int*, const int*, const double*, double*, double*);
void launch_actuation_vjp(hipStream_t, int, int, const int*, const double*, const double*, const double*,
                          const int*, const int*, const double*, double*, double*);
void launch_scatter_ht(hipStream_t, int, const int*, const int*, const int*, const int*, const double*,
                       const double*, const GmresState*, double*);
void launch_delassus(hipStream_t, int, int, const int*, const long long*, const int*, const double*,
                     double*, double*, double*, double*, unsigned*);
int y_panel_words(int);
int delassus_slices(int, int);
void launch_gj_pad(hipStream_t, int, int, double*);
void launchb_gj_pivot(hipStream_t, int, const int*, const long long*, const int*, const double*, double*, int*);
void launchb_gj_step(hipStream_t, int, const int*, int, const int4*, int, const long long*, const int*, const double*,
                     double*, const double*, double*, int*);
void launch_spmv_csr3(hipStream_t, int, const long long*, const int*, const double*, const double*,
                      long long, const double*, const GmresState*, double*);
void launch_block_jacobi(hipStream_t, int, const int*, const double*, const double*, long long, const double*,
                         const GmresState*, int, double*);
void launch_block_jacobi(hipStream_t, int, const int*, const float*, const double*, long long, const double*,
                         const GmresState*, int, double*);
void launch_spmv_tasks(hipStream_t, int, const int4*, const long long*, const int*, const double*,
                       const double*, long long, const double*, const GmresState*, double*);
void launch_spmv_tasks(hipStream_t, int, const int4*, const long long*, const int*, const float*,
                       const double*, long long, const double*, const GmresState*, double*);
void launch_bsr_spmv(hipStream_t, int, int, const int*, const int*, const float*, const double*, long long,
                     const double*, double*, long long, const GmresState*);
void launch_to_f32(hipStream_t, long long, const double*, float*);
void launch_bsr_soa(hipStream_t, long long, const double*, double*, float*);
void launch_wb_gather(hipStream_t, int, int, const int*, const int*, const int*, const double*,
                      const double*, const double*, const GmresState*, double*);
void launch_wb_lu(hipStream_t, int, int, const int*, const int*, const int*, const double*, const double*,
                  const double*, int, const double*, const GmresState*, double*, double*);
void launch_wb_lu_pipe(hipStream_t, int, int, const int*, const int*, const int*, const double*, const double*,
                       const double*, const double*, const GmresState*, double*, double*, double*, double*, unsigned*,
                       int*);
void launch_lu_pipe_init(hipStream_t, int, double*, double*, unsigned*);
void launch_sweep_parts(hipStream_t, int, int, int, const int*, const int*, const long long*, const int*,
                        const double*, const long long*, const int*, const double*, const GmresState*, double*,
                        double*);
void launch_sweep_parts(hipStream_t, int, int, int, const int*, const int*, const long long*, const int*,
                        const float*, const long long*, const int*, const float*, const GmresState*, double*,
                        double*);
void launch_lu_groups(hipStream_t, int, double*, int, int);
int lu_group_blocks();
void launch_wb_correct(hipStream_t, int, int, const int*, const int*, const int*, const double*,
                       const double*, const double*, double, const double*, const GmresState*, double*);
void launch_bsr_spmv(hipStream_t, int, int, const int*, const int*, const double*, long long, const double*, double*,
                     long long, const GmresState*);
int gm_blocks(long long, int);
int bsr_blocks(int, int);
int vec_blocks(long long);
void launch_bsr_dots(hipStream_t, int, int, const int*, const int*, const double*, long long, const double*, double*,
                     long long, const GmresState*, int, double*, double* Zb = nullptr);
void launch_bsr_dots(hipStream_t, int, int, const int*, const int*, const float*, const double*, long long,
                     const double*, double*, long long, const GmresState*, int, double*, double* Zb = nullptr);
void launch_fold_partials(hipStream_t, double*, int, const GmresState*, int);
double* launch_gj_wide(hipStream_t, int, double*, double*, double*, double*, int*);
void launch_lu_pivot0(hipStream_t, int, double*, double*, int*);
void launch_lu_colpanel(hipStream_t, int, int, double*, const double*);
void launch_lu_tiles_next(hipStream_t, int, int, double*, double*, int*);
void launch_lu_tiles_rest(hipStream_t, int, int, double*);
void launch_lu_rowpanels(hipStream_t, int, double*, const double*, int, int);
size_t gj_wide_lds_bytes();
void launch_spmv_tasks_acc(hipStream_t, int, const int4*, const long long*, const int*, const double*,
                           const double*, double, const GmresState*, double*);
void launch_gather_values(hipStream_t, long long, const long long*, const double*, double*);
void launch_spmv_tasks_acc(hipStream_t, int, const int4*, const long long*, const int*, const float*,
                           const double*, double, const GmresState*, double*);
void launch_perm_gather(hipStream_t, int, const int*, const double*, long long, const double*, const GmresState*,
                        double*);
void launch_perm_scatter(hipStream_t, int, const int*, const double*, const GmresState*, double*);
void launch_bsr_residual_dd(hipStream_t, int, const int*, const int*, const double*, const double*, const double*,
                            double*);
void launch_gm_update(hipStream_t, long long, int, double*, long long, const double*, const GmresState*,
                      const double*, int, double*, double*, int);
void launch_gm_givens(hipStream_t, GmresState*, const double*, int, double*, const double*, double*, double*,
                      double*, double*);
void launch_residual(hipStream_t, long long, const double*, double*, double*, double*, GmresState*, double*,
                     double*);
void launch_pcg_xr(hipStream_t, long long, double*, double*, const double*, const double*, const double*, int,
                   const GmresState*, const double*, double*);
void launch_dot_partials(hipStream_t, long long, const double*, const double*, const GmresState*, double*);
void launch_pcg_scalar(hipStream_t, GmresState*, const double*, int, const double*, int, const double*, int,
                       double*, int);
void launch_pcg_p(hipStream_t, long long, const double*, double*, const GmresState*, const double*);
void launch_gm_finish(hipStream_t, long long, const GmresState*, const double*, const double*,
                      const double*, const double*, long long, double*, double*);
void launch_axpy(hipStream_t, long long, double, const double*, double*);
void launch_fwd_predict(hipStream_t, int, const double*, const double*, const double*, const double*, double,
                        const double*, double*, double*);
void launch_fwd_detect(hipStream_t, int, const double*, const double*, int, const double*, int, const double*,
                       const double*, double, int*);
void launch_add_vec(hipStream_t, long long, const double*, const double*, double, double*);
void launch_scale_vec(hipStream_t, long long, const double*, double, double*);
void launch_tet_force(hipStream_t, int, const int*, const double*, const double*, const double*,
                      const double*, double, const double*, double*, int*, int);
void launch_gather_force(hipStream_t, int, const int*, const int*, const double*, const double*,
                         const double*, const double*, double*);
void launch_add_contact_vec(hipStream_t, int, const int*, const double*, double*);
void launch_gather_contact_rows(hipStream_t, int, const int*, const double*, double*);
void launch_norms(hipStream_t, long long, const double*, double*, double*);

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
  adj_tuning tune{64, 16, 8, 0, 2048, 0, 4608, 1, 0};
  int nv = 0, nt = 0, nnzb = 0, max_contacts = 0;
  int material = 0;  // adj_material of the local projection
  int nb = 0;  // bilateral bindings: vertex ids and compliances on the device
  int* d_bvid = nullptr;
  double* d_bE = nullptr;
  double* d_btarget = nullptr;  // binding targets d_b of the next forward steps [n_b][3]
  bool btarget_set = false;
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
  bool delassus_f32 = false;
  bool symmetric = true;      // Acal^T symmetric: no frictional contact, or mu = 0  // D computed on FP32 matrix cores (mixed precision)
  double* d_Pws = nullptr;    // K-slice partials of the Delassus product
  // Gauss-Jordan with the pivot lookahead (the batched step kernels on a
  // batch of one): tile list of the padded size gj_mp, scene list {0},
  // offset {0}, size {gj_mp}, two pivot slots
  int gj_mp = 0;
  // wide Gauss-Jordan (128 pivot columns per step, from the padded size
  // tune.gj_wide_min up): its pivot block and panel scratch
  double *d_gjw_P = nullptr, *d_gjw_W = nullptr;
  size_t cap_gjw_W = 0;
  // block LU (from the padded size tune.lu_min up): the inverted pivot
  // blocks; with cap_lu set, d_X holds the factors instead of the inverse
  double *d_lu_P = nullptr, *d_lu_y = nullptr;  // pivot inverses; the substitutions' second vector
  size_t cap_lu_P = 0, cap_lu_y = 0;
  // pipelined substitutions: the published values of each pass, two tickets
  double *d_lu_A0 = nullptr, *d_lu_A1 = nullptr;
  size_t cap_lu_A0 = 0, cap_lu_A1 = 0;
  unsigned* d_lu_tick = nullptr;
  bool cap_lu = false;
  int4* d_gj_tiles = nullptr;
  int* d_gj_one = nullptr;        // [0] = scene 0, [1] = padded size
  long long* d_gj_xoff = nullptr;
  double* d_gj_P = nullptr;
  size_t cap_pws = 0;
  size_t cap_ncv = 0, cap_m = 0, cap_z = 0;
  long long nnzS = 0;   // entries of S
  size_t lds_max = 0;   // bytes of LDS one block may use on the scene's device
  long long mixed_fallbacks = 0;  // mixed solves finished in FP64 (refinement stalled)
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
  double* d_Zk = nullptr;  // flexible basis: the preconditioned vectors M^-1 v_j, [R][n3]
  double *d_Vt = nullptr, *d_scale = nullptr, *d_H = nullptr, *d_cs = nullptr, *d_sn = nullptr,
         *d_g = nullptr, *d_hbuf = nullptr, *d_coef = nullptr, *d_partial = nullptr;
  size_t preg = 0;  // doubles per partial-sum region (three regions in d_partial)
  double* P1() const { return d_partial; }
  double* P2() const { return d_partial + preg; }
  double* P3() const { return d_partial + 2 * preg; }
  unsigned* d_counter = nullptr;
  GmresState* d_state = nullptr;
  GmresState* h_state = nullptr;  // pinned
  double *d_t1 = nullptr, *d_u = nullptr, *d_y = nullptr, *d_r = nullptr, *d_b = nullptr,
         *d_dz = nullptr, *d_xt = nullptr;
  // mixed precision: FP32 storage of the matrices used inside the inner solve
  float *d_Sx32 = nullptr, *d_STx32 = nullptr, *d_val32 = nullptr;
  // entry-major copy of the block values read by the Krylov products
  // (d_valT[k nnzb + p] = d_val[9 p + k]; d_val32 holds the same order in FP32)
  double* d_valT = nullptr;
  bool mixed_ready = false;
  // forward step
  double* d_planes = nullptr;
  // kinematic spheres of the next forward step: [old pose][new pose], each
  // n_spheres x (centre, radius), host copy and device copy
  // Woodbury correction through the cached Z (use_z) or through S^T S with
  // the scatter buffer d_wz and the product d_wz2 ([3 n_v] each)
  bool use_z = true, z_built = false;
  double *d_wz = nullptr, *d_wz2 = nullptr;
  // Without Z the correction is applied through Y = S E (the columns of S at
  // the contact vertices, CSR by elimination row; columns are vertex ids):
  // one S and one S^T product per apply plus two products with Y.  Tasks of
  // the Y rows with entries, and of the contact-vertex rows of S^T.
  char* h_ystage = nullptr;  // pinned staging of the Y row lists
  size_t cap_ystage = 0;
  long long *d_Yp = nullptr, *d_Ysrc = nullptr;
  int *d_Ycol = nullptr, *d_Ytasks = nullptr, *d_CTtasks = nullptr;
  double* d_Yval = nullptr;
  int nY_tasks = 0, nCT_tasks = 0;
  size_t cap_ynnz = 0, cap_ytasks = 0, cap_cttasks = 0;
  long long y_nnz = 0;
  unsigned* d_ybm = nullptr;  // panel occupancy of Y for the Delassus product
  size_t cap_ybm = 0;
  // A^{-1} through level-scheduled sweeps with L instead of the S products
  // (use_sweeps, from tune.a_inv): device copies of the host sweep arrays
  // (FP64 and FP32 values), the permutation, two work vectors [3 n_v]
  bool sweeps_built = false, use_sweeps = false;
  int n_levels = 0;
  long long *d_Fp = nullptr, *d_Bp = nullptr, *d_Ip = nullptr, *d_ITp = nullptr;
  int *d_Fj = nullptr, *d_Bj = nullptr, *d_Ij = nullptr, *d_ITj = nullptr, *d_perm = nullptr;
  double *d_Fx = nullptr, *d_Bx = nullptr, *d_Ix = nullptr, *d_ITx = nullptr, *d_lt = nullptr, *d_lz = nullptr;
  float *d_Fx32 = nullptr, *d_Bx32 = nullptr, *d_Ix32 = nullptr, *d_ITx32 = nullptr;
  int *d_fA = nullptr, *d_fB = nullptr, *d_bA = nullptr, *d_bB = nullptr;
  // the lowest fuse_k levels of each sweep in one launch (k_sweep_parts):
  // n_parts independent parts, their rows and per-height offsets
  int fuse_k = 0, n_parts = 0;
  int *d_part_rows = nullptr, *d_part_off = nullptr;
  // actuation (active stress per tet group): group and fibre per tet, the
  // tets of each group (CSR), per-tet scratch
  int n_act = 0;
  int *d_act_group = nullptr, *d_act_gptr = nullptr, *d_act_gtets = nullptr;
  double *d_act_fibre = nullptr, *d_act12 = nullptr, *d_act_s = nullptr;
  int n_spheres = 0, sph_cap = 0;  // sph_cap: spheres d_sph has room for
  std::vector<double> sph;
  double* d_sph = nullptr;
  int *d_vptr = nullptr, *d_vcode = nullptr, *d_mask = nullptr, *d_fvid = nullptr;
  double *d_force = nullptr, *d_utilde = nullptr, *d_qtilde = nullptr, *d_fu = nullptr, *d_du = nullptr,
         *d_ut = nullptr, *d_qcur = nullptr, *d_rq = nullptr, *d_rhs = nullptr, *d_cvec = nullptr,
         *d_cu = nullptr, *d_norms = nullptr, *d_x_pcg = nullptr;
  std::unordered_map<long long, std::pair<double, double>> warm;
  int fwd_newton_iters = 0;
  double fwd_residual = 0.0;
  // captured Krylov chunks (tuning.graph = 1), rebuilt after every setup
  hipStream_t cap_stream = nullptr;
  // second stream of the block-LU factorisation (the bulk of each trailing
  // update runs there beside the next panel and its pivot inversion) and its
  // two ordering events; default priority
  hipStream_t lu_stream = nullptr, lu_post_stream = nullptr;
  hipEvent_t lu_ev[3] = {nullptr, nullptr, nullptr};
  hipGraphExec_t chunk_exec[8] = {};  // [pcg][FP32 preconditioner][FP32 product]
  // preconditioner of the Krylov solves (adj_precond), set per solve;
  // woodbury_ready: the last setup built the capacitance inverse
  int precond = ADJ_PRECOND_WOODBURY;
  bool woodbury_ready = false;
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
      // device-scope events: no system-scope cache fence around the timed
      // launch (the timing brackets only work on this device)
      hipEvent_t a, b;
      if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess) return;
      if (hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess) {
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
                  s->d_colbuf,   s->d_tvec,   s->d_Vt,    s->d_Zk,  s->d_scale,       s->d_H,
                  s->d_cs,       s->d_sn,     s->d_g,     s->d_hbuf,        s->d_coef,
                  s->d_partial,  s->d_counter, s->d_state, s->d_t1,         s->d_u,
                  s->d_y,        s->d_r,      s->d_b,     s->d_dz,          s->d_xt,
                  s->d_Stasks,   s->d_STtasks, s->d_planes,  s->d_vptr,   s->d_vcode, s->d_sph,
                  s->d_wz,       s->d_wz2,    s->d_gj_tiles, s->d_gj_one, s->d_gj_xoff, s->d_gj_P,
                  s->d_act_group, s->d_act_gptr, s->d_act_gtets, s->d_act_fibre, s->d_act12, s->d_act_s,
                  s->d_mask,     s->d_fvid,   s->d_force, s->d_utilde,      s->d_qtilde,
                  s->d_fu,       s->d_du,     s->d_ut,    s->d_qcur,        s->d_rq,
                  s->d_rhs,      s->d_cvec,   s->d_cu,    s->d_norms,       s->d_Sx32,
                  s->d_STx32,    s->d_val32,  s->d_valT,  s->d_Pws,   s->d_x_pcg, s->d_bvid, s->d_bE, s->d_btarget,
                  s->d_Yp,       s->d_Ysrc,   s->d_Ycol,  s->d_Ytasks,      s->d_CTtasks, s->d_Yval,
                  s->d_gjw_P,    s->d_gjw_W,  s->d_lu_P,  s->d_lu_y, s->d_lu_A0, s->d_lu_A1, s->d_lu_tick,
                  s->d_Fp, s->d_Bp, s->d_Ip, s->d_ITp, s->d_Fj, s->d_Bj, s->d_Ij, s->d_ITj, s->d_perm,
                  s->d_Fx, s->d_Bx, s->d_Ix, s->d_ITx, s->d_lt, s->d_lz, s->d_Fx32, s->d_Bx32, s->d_Ix32, s->d_ITx32,
                  s->d_fA, s->d_fB, s->d_bA, s->d_bB, s->d_ybm, s->d_part_rows, s->d_part_off};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (s->h_state) (void)hipHostFree(s->h_state);
  if (s->h_ystage) (void)hipHostFree(s->h_ystage);
  for (hipEvent_t e : s->prof_ev) (void)hipEventDestroy(e);
  for (hipGraphExec_t& g : s->chunk_exec)
    if (g) (void)hipGraphExecDestroy(g);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  for (hipEvent_t e : s->lu_ev)
    if (e) (void)hipEventDestroy(e);
  if (s->lu_stream) (void)hipStreamDestroy(s->lu_stream);
  if (s->lu_post_stream) (void)hipStreamDestroy(s->lu_post_stream);
  delete s;
}

static const int kMaxRestart = 128;
// Relative residual below which plain FP64 Krylov solves stagnate on stiff
// contact states; FP64 solves asked for less (with max_refine > 0) refine
// with a double-double residual.
static const double kFp64Floor = 1e-9;

extern "C" const char* adj_last_error(void) { return g_err.c_str(); }

// Largest contact count of one scene: m = 3 n_c <= 30000 keeps the padded
// capacitance (mp^2 entries) addressable with 32-bit offsets.
constexpr int kMaxContacts = 10000;

// Scene construction without the per-scene contact cap (a batch's union
// scene holds the sum of its scenes' contacts; its capacitance stays per
// scene).
static adj_status scene_create(const adj_scene_desc* desc, int32_t max_contacts, adj_scene** out);

// Levels of each sweep run as one launch (k_sweep_parts): tune.sweep_fuse
// levels, or with -1 the most levels that still split into at least 256
// independent parts (one block each); 0 or no sweeps: none.  Rebuilds the
// device lists when the count changes (synchronous; not inside a capture).
static adj_status prepare_sweep_parts(adj_scene* s) {
  if (!s->sweeps_built) return ADJ_OK;
  int k = s->tune.sweep_fuse;
  std::vector<int32_t> rows, off;
  if (k < 0) {
    k = 0;
    for (int c = 1; c < s->n_levels; ++c) {
      if (sweep_parts(s->hs, c, rows, off) < 256) break;
      k = c;
    }
  }
  k = std::min(k, s->n_levels);
  if (k == s->fuse_k && (k == 0 || s->d_part_rows)) return ADJ_OK;
  (void)hipFree(s->d_part_rows);
  (void)hipFree(s->d_part_off);
  s->d_part_rows = s->d_part_off = nullptr;
  s->fuse_k = s->n_parts = 0;
  if (k == 0) return ADJ_OK;
  const int np = sweep_parts(s->hs, k, rows, off);
  if (np <= 0) return ADJ_OK;
  if (dalloc(&s->d_part_rows, std::max<size_t>(rows.size(), 1)) != hipSuccess ||
      dalloc(&s->d_part_off, off.size()) != hipSuccess)
    return fail(ADJ_E_OOM, "hipMalloc failed (sweep parts)");
  if (hipMemcpy(s->d_part_rows, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(s->d_part_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
    return fail(ADJ_E_DEVICE, "hipMemcpy failed (sweep parts)");
  s->fuse_k = k;
  s->n_parts = np;
  return ADJ_OK;
}

extern "C" adj_status adj_scene_create(const adj_scene_desc* desc, int32_t max_contacts,
                                       adj_scene** out) {
  if (!out) return fail(ADJ_E_ARG, "out is null");
  *out = nullptr;
  if (max_contacts > kMaxContacts) return fail(ADJ_E_ARG, "max_contacts above 10000");
  return scene_create(desc, max_contacts, out);
}

static adj_status scene_create(const adj_scene_desc* desc, int32_t max_contacts, adj_scene** out) {
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
  s->nnzS = (long long)h.Sj.size();
  {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds <= 0) {
      free_scene(s);
      return fail(ADJ_E_DEVICE, "cannot query the device's LDS size");
    }
    s->lds_max = (size_t)lds;
  }
#define UP(dst, src)                                   \
  do {                                                 \
    hipError_t e_ = upload(&dst, src);                 \
    if (e_ != hipSuccess) {                            \
      free_scene(s);                                   \
      return fail(ADJ_E_OOM, "device upload failed");  \
    }                                                  \
  } while (0)
  std::vector<long long> Sp(h.Sp.begin(), h.Sp.end()), STp(h.STp.begin(), h.STp.end());
  // per-tet arrays entry-major on the device (entry e of tet t at e * n_t + t), so that the per-tet
  // kernels' loads coalesce: the four vertex ids and the 12 entries of B~ per tet
  auto entry_major = [&](const auto& v, int w) {
    std::remove_const_t<std::remove_reference_t<decltype(v)>> out(v.size());
    for (int t = 0; t < h.nt; ++t)
      for (int e = 0; e < w; ++e) out[(size_t)e * h.nt + t] = v[(size_t)t * w + e];
    return out;
  };
  UP(s->d_tets, entry_major(h.tets, 4));
  UP(s->d_rowptr, h.rowptr);
  UP(s->d_col, h.col);
  UP(s->d_row_of_slot, h.row_of_slot);
  UP(s->d_diag_slot, h.diag_slot);
  s->nb = (int)h.bvid.size();
  s->material = h.material;
  if (s->nb) {
    UP(s->d_bvid, h.bvid);
    UP(s->d_bE, h.bE);
    UP(s->d_btarget, std::vector<double>(3 * h.bvid.size(), 0.0));
  }
  UP(s->d_slot_ptr, h.slot_ptr);
  UP(s->d_slot_code, h.slot_code);
  UP(s->d_Bt, entry_major(h.Bt, 12));
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
  UP(s->d_planes, h.planes);
  UP(s->d_vptr, h.vptr);
  UP(s->d_vcode, h.vcode);
  UP(s->d_Stasks, h.S_tasks);
  UP(s->d_STtasks, h.ST_tasks);
  s->nS_tasks = (int)(h.S_tasks.size() / 4);
  s->nST_tasks = (int)(h.ST_tasks.size() / 4);
  if (h.n_levels > 0) {
    std::vector<long long> Fp(h.Fp.begin(), h.Fp.end()), Bp(h.Bp.begin(), h.Bp.end()),
        Ip(h.Ip.begin(), h.Ip.end()), ITp(h.ITp.begin(), h.ITp.end());
    UP(s->d_Fp, Fp);
    UP(s->d_Bp, Bp);
    UP(s->d_Ip, Ip);
    UP(s->d_ITp, ITp);
    UP(s->d_Fj, h.Fj);
    UP(s->d_Bj, h.Bj);
    UP(s->d_Ij, h.Ij);
    UP(s->d_ITj, h.ITj);
    UP(s->d_Fx, h.Fx);
    UP(s->d_Bx, h.Bx);
    UP(s->d_Ix, h.Ix);
    UP(s->d_ITx, h.ITx);
    UP(s->d_perm, h.perm);
    UP(s->d_fA, h.fA_tasks);
    UP(s->d_fB, h.fB_tasks);
    UP(s->d_bA, h.bA_tasks);
    UP(s->d_bB, h.bB_tasks);
    s->n_levels = h.n_levels;
    s->sweeps_built = true;
  }
#undef UP
  bool ok = true;
  const size_t mc = (size_t)std::max(1, max_contacts);
  const size_t R = kMaxRestart;
  // per-block partial sums: enough blocks for any tuning (block-sparse
  // product with 32 lanes per row, Gram-Schmidt with 64 rows per block,
  // vector kernels with at most 512 blocks)
  const size_t nblk = std::max<size_t>({(size_t)bsr_blocks(s->nv, 32), (size_t)gm_blocks(s->n3, 64), 512}) + 8;
  s->preg = nblk * 130;
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
  ok &= dalloc(&s->d_tvec, (3 * mc + 127) / 128 * 128) == hipSuccess;  // padded: block-LU substitutions
  ok &= dalloc(&s->d_P, 32 * 32) == hipSuccess;
  ok &= dalloc(&s->d_Vt, (R + 1) * (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_Zk, R * (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_scale, R + 2) == hipSuccess;
  ok &= dalloc(&s->d_H, (R + 1) * R) == hipSuccess;
  ok &= dalloc(&s->d_cs, R + 1) == hipSuccess;
  ok &= dalloc(&s->d_sn, R + 1) == hipSuccess;
  ok &= dalloc(&s->d_g, R + 2) == hipSuccess;
  ok &= dalloc(&s->d_hbuf, 260) == hipSuccess;
  ok &= dalloc(&s->d_coef, 130) == hipSuccess;
  ok &= dalloc(&s->d_partial, 3 * s->preg) == hipSuccess;
  ok &= dalloc(&s->d_counter, 16) == hipSuccess;
  ok &= dalloc(&s->d_state, 1) == hipSuccess;
  ok &= dalloc(&s->d_t1, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_u, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_y, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_r, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_b, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_dz, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_xt, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_x_pcg, (size_t)s->n3) == hipSuccess;
  ok &= hipHostMalloc((void**)&s->h_state, sizeof(GmresState), hipHostMallocDefault) == hipSuccess;
  ok &= dalloc(&s->d_mask, (size_t)s->nv) == hipSuccess;
  ok &= dalloc(&s->d_Sx32, h.Sx.size()) == hipSuccess;
  ok &= dalloc(&s->d_STx32, h.STx.size()) == hipSuccess;
  ok &= dalloc(&s->d_val32, 9 * (size_t)s->nnzb) == hipSuccess;
  ok &= dalloc(&s->d_valT, 9 * (size_t)s->nnzb) == hipSuccess;
  ok &= dalloc(&s->d_fvid, mc) == hipSuccess;
  ok &= dalloc(&s->d_force, 12 * (size_t)s->nt) == hipSuccess;
  ok &= dalloc(&s->d_utilde, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_qtilde, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_fu, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_du, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_ut, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_qcur, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_rq, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_rhs, (size_t)s->n3) == hipSuccess;
  ok &= dalloc(&s->d_cvec, 3 * mc) == hipSuccess;
  ok &= dalloc(&s->d_cu, 3 * mc) == hipSuccess;
  ok &= dalloc(&s->d_norms, 4) == hipSuccess;
  if (!ok) {
    free_scene(s);
    return fail(ADJ_E_OOM, "device workspace allocation failed");
  }
  if (s->sweeps_built) {
    ok &= dalloc(&s->d_lt, (size_t)s->n3) == hipSuccess;
    ok &= dalloc(&s->d_lz, (size_t)s->n3) == hipSuccess;
    ok &= dalloc(&s->d_Fx32, std::max<size_t>(h.Fx.size(), 1)) == hipSuccess;
    ok &= dalloc(&s->d_Bx32, std::max<size_t>(h.Bx.size(), 1)) == hipSuccess;
    ok &= dalloc(&s->d_Ix32, std::max<size_t>(h.Ix.size(), 1)) == hipSuccess;
    ok &= dalloc(&s->d_ITx32, std::max<size_t>(h.ITx.size(), 1)) == hipSuccess;
    if (!ok) {
      free_scene(s);
      return fail(ADJ_E_OOM, "device workspace allocation failed (sweeps)");
    }
    launch_to_f32(nullptr, (long long)h.Fx.size(), s->d_Fx, s->d_Fx32);
    launch_to_f32(nullptr, (long long)h.Bx.size(), s->d_Bx, s->d_Bx32);
    launch_to_f32(nullptr, (long long)h.Ix.size(), s->d_Ix, s->d_Ix32);
    launch_to_f32(nullptr, (long long)h.ITx.size(), s->d_ITx, s->d_ITx32);
  }
  launch_to_f32(nullptr, (long long)h.Sx.size(), s->d_Sx, s->d_Sx32);
  launch_to_f32(nullptr, (long long)h.STx.size(), s->d_STx, s->d_STx32);
  if (prepare_sweep_parts(s) != ADJ_OK) {
    free_scene(s);
    return fail(ADJ_E_OOM, "device workspace allocation failed (sweep parts)");
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
  if (*p) {
    (void)hipDeviceSynchronize();  // the old buffer may still be read on another stream
    (void)hipFree(*p);
  }
  *p = nullptr;
  if (dalloc(p, need) != hipSuccess) {
    *cap = 0;
    return fail(ADJ_E_OOM, "device allocation failed");
  }
  *cap = need;
  return ADJ_OK;
}

// Contact bookkeeping shared by the adjoint and the forward step: unique
// contact vertices, capacitance row layout, upload of the maps, and the
static void drop_chunk_graphs(adj_scene* s) {
  for (hipGraphExec_t& g : s->chunk_exec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Delassus matrix / Z (rebuilt only when the contact vertex set changes).
// Forming Z = S^T (S E) costs nnz(S) x n_cv multiply-adds; above this the
// Woodbury correction goes through S^T S at every apply instead.
static const double kZBudget = 2e10;

// Y = S E as CSR by elimination row (the correction without Z): column k of
// Y is the column of S at contact vertex cv[k], i.e. row cv[k] of S^T, which
// is nonzero exactly on the elimination-tree path from that vertex to the
// root.  Rows list their contact vertices in increasing k (vertex order);
// values are gathered on the device from S^T.  Also the task list of the
// contact-vertex rows of S^T (the contact entries of A^{-1} r).
static adj_status int_upload(int** p, size_t* cap, const std::vector<int32_t>& v, hipStream_t st) {
  if (v.size() > *cap || !*p) {
    if (*p) {
      (void)hipDeviceSynchronize();
      (void)hipFree(*p);
    }
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(p, std::max<size_t>(v.size(), 1) * sizeof(int)) != hipSuccess) return fail(ADJ_E_OOM, "tasks");
    *cap = v.size();
  }
  if (!v.empty()) HIPCHK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, st));
  return ADJ_OK;
}

static adj_status build_y_rows(adj_scene* s, hipStream_t st, const std::vector<int>& cv) {
  const HostScene& h = s->hs;
  const int nv = s->nv, ncv = (int)cv.size();
  // host threads over contiguous ranges of contact vertices (balanced by
  // path length): per-thread row counts, then each thread fills its rows'
  // entries from its own cursors, so every row lists its contact vertices
  // in increasing k exactly as one thread would
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<int> kb(nth + 1, ncv);
  {
    long long total = 0;
    for (int k = 0; k < ncv; ++k) total += h.STp[cv[k] + 1] - h.STp[cv[k]];
    long long acc = 0;
    int t = 1;
    kb[0] = 0;
    for (int k = 0; k < ncv && t < nth; ++k) {
      acc += h.STp[cv[k] + 1] - h.STp[cv[k]];
      while (t < nth && acc * nth >= total * t) kb[t++] = k + 1;
    }
  }
  std::vector<std::vector<int64_t>> cur(nth, std::vector<int64_t>(nv + 1, 0));
  auto run = [&](auto&& body) {
    std::vector<std::thread> pool;
    for (int t = 1; t < nth; ++t) pool.emplace_back(body, t);
    body(0);
    for (auto& th : pool) th.join();
  };
  run([&](int t) {
    std::vector<int64_t>& c = cur[t];
    for (int k = kb[t]; k < kb[t + 1]; ++k)
      for (int64_t p = h.STp[cv[k]]; p < h.STp[cv[k] + 1]; ++p) c[h.STj[p]]++;
  });
  std::vector<int64_t> yp(nv + 1, 0);
  for (int r = 0; r < nv; ++r) {
    int64_t o = yp[r];
    for (int t = 0; t < nth; ++t) {
      const int64_t n = cur[t][r];
      cur[t][r] = o;  // thread t's cursor in row r
      o += n;
    }
    yp[r + 1] = o;
  }
  const long long nnz = yp[nv];
  // pinned staging of the column and source lists (kept by the scene)
  const size_t need = (size_t)std::max<long long>(nnz, 1) * (sizeof(int32_t) + sizeof(int64_t));
  if (need > s->cap_ystage) {
    if (s->h_ystage) (void)hipHostFree(s->h_ystage);
    s->h_ystage = nullptr;
    s->cap_ystage = 0;
    if (hipHostMalloc((void**)&s->h_ystage, need, hipHostMallocDefault) != hipSuccess)
      return fail(ADJ_E_OOM, "pinned staging of the Y rows");
    s->cap_ystage = need;
  }
  int64_t* ysrc = reinterpret_cast<int64_t*>(s->h_ystage);
  int32_t* ycol = reinterpret_cast<int32_t*>(s->h_ystage + (size_t)std::max<long long>(nnz, 1) * sizeof(int64_t));
  run([&](int t) {
    std::vector<int64_t>& c = cur[t];
    for (int k = kb[t]; k < kb[t + 1]; ++k)
      for (int64_t p = h.STp[cv[k]]; p < h.STp[cv[k] + 1]; ++p) {
        const int64_t o = c[h.STj[p]]++;
        ycol[o] = cv[k];
        ysrc[o] = p;
      }
  });
  const std::vector<int32_t> ytasks = make_row_tasks(yp, 1024, nullptr, true);
  std::vector<int32_t> rows(cv.begin(), cv.end());
  const std::vector<int32_t> cttasks = make_row_tasks(h.STp, 1024, &rows);
  if ((size_t)nnz > s->cap_ynnz || !s->d_Ycol) {
    (void)hipDeviceSynchronize();
    for (void* p : {(void*)s->d_Ycol, (void*)s->d_Ysrc, (void*)s->d_Yval})
      if (p) (void)hipFree(p);
    s->d_Ycol = nullptr;
    s->d_Ysrc = nullptr;
    s->d_Yval = nullptr;
    s->cap_ynnz = 0;
    const size_t n = std::max<long long>(nnz, 1);
    if (hipMalloc(&s->d_Ycol, n * sizeof(int)) != hipSuccess ||
        hipMalloc(&s->d_Ysrc, n * sizeof(long long)) != hipSuccess ||
        hipMalloc(&s->d_Yval, n * sizeof(double)) != hipSuccess)
      return fail(ADJ_E_OOM, "Y rows of the Woodbury correction");
    s->cap_ynnz = nnz;
  }
  if (!s->d_Yp && hipMalloc(&s->d_Yp, (size_t)(nv + 1) * sizeof(long long)) != hipSuccess)
    return fail(ADJ_E_OOM, "Y row pointer");
  HIPCHK(hipMemcpyAsync(s->d_Yp, yp.data(), (nv + 1) * sizeof(long long), hipMemcpyHostToDevice, st));
  if (nnz) {
    HIPCHK(hipMemcpyAsync(s->d_Ycol, ycol, nnz * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_Ysrc, ysrc, nnz * sizeof(long long), hipMemcpyHostToDevice, st));
  }
  adj_status a;
  if ((a = int_upload(&s->d_Ytasks, &s->cap_ytasks, ytasks, st)) != ADJ_OK) return a;
  if ((a = int_upload(&s->d_CTtasks, &s->cap_cttasks, cttasks, st)) != ADJ_OK) return a;
  launch_gather_values(st, nnz, s->d_Ysrc, s->d_STx, s->d_Yval);
  HIPCHK(hipStreamSynchronize(st));  // the host vectors go out of scope, the staging is reused
  s->nY_tasks = (int)(ytasks.size() / 4);
  s->nCT_tasks = (int)(cttasks.size() / 4);
  s->y_nnz = nnz;
  return ADJ_OK;
}

static adj_status contact_layout(adj_scene* s, hipStream_t st, int nc, const std::vector<int>& vid,
                                 const std::vector<int>& fric, bool reuse, bool delassus = true,
                                 bool force_no_z = false) {
  drop_chunk_graphs(s);  // captured chunks hold the contact layout
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
  if (nc) {
    HIPCHK(hipMemcpyAsync(s->d_cmap, cmap.data(), nc * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_c_row0, c_row0.data(), nc * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_c_nrow, c_nrow.data(), nc * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_row_c, row_c.data(), m * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_row_i, row_i.data(), m * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_cv, cv.data(), ncv * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_cv_ptr, cv_ptr.data(), (ncv + 1) * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));  // host vectors go out of scope
  }
  s->delassus_rebuilt = 0;
  const bool use_z = !force_no_z && (double)s->nnzS * (double)ncv <= kZBudget;
  if (nc && delassus && !(reuse && s->delassus_valid && cv == s->cv_cached && (s->z_built || !use_z))) {
    adj_status a;
    // the Woodbury kernels stage m (gather) and 3 n_cv (Z correction)
    // doubles in LDS
    if ((size_t)8 * m > s->lds_max || (use_z && (size_t)24 * ncv > s->lds_max))
      return fail(ADJ_E_SHAPE, "capacitance or contact-vertex count beyond the LDS staging of the Woodbury kernels");
    size_t capY = s->cap_ncv ? (size_t)s->nv * s->cap_ncv : 0, capD = s->cap_ncv * s->cap_ncv;
    size_t capZ = s->cap_z;
    if ((size_t)ncv > s->cap_ncv) capY = capD = 0;
    if ((a = grow(&s->d_Y, &capY, (size_t)s->nv * ncv)) != ADJ_OK) return a;
    if ((a = grow(&s->d_D, &capD, (size_t)ncv * ncv)) != ADJ_OK) return a;
    if (use_z && (a = grow(&s->d_Z, &capZ, (size_t)s->nv * ncv)) != ADJ_OK) return a;
    s->cap_z = capZ;
    s->cap_ncv = std::max(s->cap_ncv, (size_t)ncv);
    if (!use_z) {
      size_t cw = s->d_wz ? (size_t)s->n3 : 0, cw2 = cw;
      if ((a = grow(&s->d_wz, &cw, (size_t)s->n3)) != ADJ_OK) return a;
      if ((a = grow(&s->d_wz2, &cw2, (size_t)s->n3)) != ADJ_OK) return a;
    }
    const int ks = delassus_slices(s->nv, ncv);
    if (ks > 1 && (a = grow(&s->d_Pws, &s->cap_pws, (size_t)ks * ncv * ncv)) != ADJ_OK) return a;
    {
      ProfScope p(s, 11, st);
      const size_t nbm = (size_t)((ncv + 63) / 64) * y_panel_words(s->nv);
      if (nbm > s->cap_ybm) {
        (void)hipDeviceSynchronize();
        if (s->d_ybm) (void)hipFree(s->d_ybm);
        s->d_ybm = nullptr;
        s->cap_ybm = 0;
        if (hipMalloc(&s->d_ybm, nbm * sizeof(unsigned)) != hipSuccess) return fail(ADJ_E_OOM, "Y panel bitmap");
        s->cap_ybm = nbm;
      }
      launch_delassus(st, s->nv, ncv, s->d_cv, s->d_STp, s->d_STj, s->d_STx, s->d_Y, s->d_D,
                      use_z ? s->d_Z : nullptr, s->d_Pws, s->d_ybm);
    }
    if (!use_z && (a = build_y_rows(s, st, cv)) != ADJ_OK) return a;
    s->cv_cached = cv;
    s->delassus_valid = true;
    s->delassus_rebuilt = 1;
    s->z_built = use_z;
  }
  s->use_z = use_z;
  return ADJ_OK;
}

// Capacitance Khat^{-T} + h^2 Hq A^{-1} Hq^T (transpose = 1, adjoint) or
// Khat^{-1} + ... (transpose = 0, forward Newton) from s->d_Q, s->d_kh, and
// its inverse s->d_X.
static adj_status build_capacitance(adj_scene* s, hipStream_t st, double mu, int transpose) {
  drop_chunk_graphs(s);  // captured chunks hold the contact layout and the address of X
  if (!s->nc) return ADJ_OK;
  const double h2 = s->hs.h * s->hs.h;
  const int m = s->m;
  if (m > 3 * kMaxContacts) return fail(ADJ_E_SHAPE, "more than 10000 contacts in one capacitance");
  // narrow Gauss-Jordan tiles are 64 x 64, the wide steps 128 columns
  const int mpw = ((m + 127) / 128) * 128;
  const bool big_lds = s->lds_max >= gj_wide_lds_bytes();
  const bool lu = mpw >= s->tune.lu_min && big_lds;
  const bool wide = lu || (mpw >= s->tune.gj_wide_min && big_lds);
  const int mp = wide ? mpw : ((m + 63) / 64) * 64;
  s->mp = mp;
  s->cap_lu = lu;
  size_t capC = s->cap_m * s->cap_m, capB = capC;
  if ((size_t)mp > s->cap_m) capC = capB = 0;
  adj_status a;
  if ((a = grow(&s->d_C, &capC, (size_t)mp * mp)) != ADJ_OK) return a;
  if ((a = grow(&s->d_colbuf, &capB, (size_t)mp * mp)) != ADJ_OK) return a;
  s->cap_m = std::max(s->cap_m, (size_t)mp);
  launch_capacitance(st, m, mp, s->d_row_c, s->d_row_i, s->d_cmap, s->ncv, s->d_D, s->d_Q, s->d_kh, mu, h2,
                     transpose, s->d_C);
  if (lu) {
    if ((a = grow(&s->d_lu_P, &s->cap_lu_P, (size_t)mp * 128)) != ADJ_OK) return a;
    if ((a = grow(&s->d_lu_y, &s->cap_lu_y, (size_t)mp)) != ADJ_OK) return a;
    if ((a = grow(&s->d_lu_A0, &s->cap_lu_A0, (size_t)mp)) != ADJ_OK) return a;
    if ((a = grow(&s->d_lu_A1, &s->cap_lu_A1, (size_t)mp)) != ADJ_OK) return a;
    if (!s->d_lu_tick && dalloc(&s->d_lu_tick, 2) != hipSuccess) return fail(ADJ_E_OOM, "hipMalloc failed");
    ProfScope p(s, 7, st);
    launch_gj_pad(st, m, mp, s->d_C);
    if (!s->lu_stream && hipStreamCreateWithFlags(&s->lu_stream, hipStreamNonBlocking) != hipSuccess)
      return fail(ADJ_E_DEVICE, "hipStreamCreateWithFlags failed");
    if (!s->lu_post_stream && hipStreamCreateWithFlags(&s->lu_post_stream, hipStreamNonBlocking) != hipSuccess)
      return fail(ADJ_E_DEVICE, "hipStreamCreateWithFlags failed");
    for (hipEvent_t& e : s->lu_ev)
      if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return fail(ADJ_E_DEVICE, "hipEventCreateWithFlags failed");
    hipEvent_t e_cp = s->lu_ev[0], e_rest = s->lu_ev[1], e_post = s->lu_ev[2];
    const hipStream_t sq[2] = {st, s->lu_stream}, sx = s->lu_post_stream;
    const int nbk = mp / 128, gb = lu_group_blocks();
    // Row panels V_Kj = P_k A_Kj and the group rewrites of the factors for the
    // substitutions: a step's row panel is final once its next column and
    // bulk have run, a group's blocks once its last step has, and neither is
    // read by a later step.  From the step where the trailing matrix is down
    // to 24 blocks (the bulk no longer fills the chip and the steps wait on
    // the pivot chain) those of the finished steps run on a third stream beside
    // the chain; the rest after the last step.
    const int k_post = std::max(1, nbk - 25);
    int k_rp = 0, g_done = 0;
    bool posted = false;
    launch_lu_pivot0(st, mp, s->d_C, s->d_lu_P, s->d_err);
    if (nbk > 1) launch_lu_colpanel(st, mp, 0, s->d_C, s->d_lu_P);
    HIPCHK(hipEventRecord(e_cp, st));
    // Per step k the two streams swap roles.  The bulk of the trailing update
    // runs on sq[k % 2], behind the column panel of step k (same stream) and
    // the bulk of step k - 1 (event).  The next panel's column with the next
    // pivot inverse, then the next column panel, run on sq[(k + 1) % 2]
    // directly behind the bulk of step k - 1 in that stream, so that they are
    // released before the bulk of step k (which waits on an event) and their
    // blocks, which need a whole CU each, are placed first.
    for (int k = 0; k + 1 < nbk; ++k) {
      const hipStream_t sa = sq[k & 1], sn = sq[(k + 1) & 1];
      if (k >= k_post && (k > k_rp || k / gb > g_done)) {
        // steps < k are finished once the bulk of step k - 1 and the next
        // column of step k - 1 (with the column panel of step k) are
        HIPCHK(hipStreamWaitEvent(sx, e_rest, 0));
        HIPCHK(hipStreamWaitEvent(sx, e_cp, 0));
        launch_lu_rowpanels(sx, mp, s->d_C, s->d_lu_P, k_rp, k);
        launch_lu_groups(sx, mp, s->d_C, g_done, k / gb);
        HIPCHK(hipEventRecord(e_post, sx));
        k_rp = k;
        g_done = k / gb;
        posted = true;
      }
      HIPCHK(hipStreamWaitEvent(sn, e_cp, 0));  // the column panel of step k
      launch_lu_tiles_next(sn, mp, k, s->d_C, s->d_lu_P, s->d_err);
      if (k + 2 < nbk) launch_lu_colpanel(sn, mp, k + 1, s->d_C, s->d_lu_P);
      HIPCHK(hipEventRecord(e_cp, sn));
      if (k > 0) HIPCHK(hipStreamWaitEvent(sa, e_rest, 0));  // the bulk of step k - 1
      {
        ProfScope pk(s, 12, sa);
        launch_lu_tiles_rest(sa, mp, k, s->d_C);
      }
      HIPCHK(hipEventRecord(e_rest, sa));
    }
    if (nbk > 1) {
      HIPCHK(hipStreamWaitEvent(st, e_cp, 0));
      HIPCHK(hipStreamWaitEvent(st, e_rest, 0));
    }
    if (posted) HIPCHK(hipStreamWaitEvent(st, e_post, 0));
    launch_lu_rowpanels(st, mp, s->d_C, s->d_lu_P, k_rp, nbk);
    launch_lu_groups(st, mp, s->d_C, g_done, nbk);
    s->d_X = s->d_C;
    // the substitutions run over all mp rows: the padding rows of t stay zero
    launch_fill_zero(st, (size_t)(mp - m), s->d_tvec + m);
    launch_lu_pipe_init(st, mp, s->d_lu_A0, s->d_lu_A1, s->d_lu_tick);
    return ADJ_OK;
  }
  if (wide) {
    size_t capP = s->d_gjw_P ? (size_t)128 * 128 : 0;
    if ((a = grow(&s->d_gjw_P, &capP, (size_t)128 * 128)) != ADJ_OK) return a;
    if ((a = grow(&s->d_gjw_W, &s->cap_gjw_W, (size_t)mp * 128)) != ADJ_OK) return a;
    ProfScope p(s, 7, st);
    launch_gj_pad(st, m, mp, s->d_C);
    s->d_X = launch_gj_wide(st, mp, s->d_C, s->d_colbuf, s->d_gjw_P, s->d_gjw_W, s->d_err);
    return ADJ_OK;
  }
  if (mp != s->gj_mp) {
    // tiles {scene 0, I, J} of the padded matrix, the same at every step
    const int nt = mp / 64;
    std::vector<int4> tiles((size_t)nt * nt);
    for (int i = 0; i < nt; ++i)
      for (int j = 0; j < nt; ++j) tiles[(size_t)i * nt + j] = make_int4(0, i, j, 0);
    const int one[2] = {0, mp};
    const long long zero = 0;
    HIPCHK(hipStreamSynchronize(st));  // the previous tile list may still be read
    for (void* p : {(void*)s->d_gj_tiles, (void*)s->d_gj_one, (void*)s->d_gj_xoff, (void*)s->d_gj_P})
      if (p) HIPCHK(hipFree(p));
    s->d_gj_tiles = nullptr;
    s->d_gj_one = nullptr;
    s->d_gj_xoff = nullptr;
    s->d_gj_P = nullptr;
    s->gj_mp = 0;
    if (hipMalloc(&s->d_gj_tiles, tiles.size() * sizeof(int4)) != hipSuccess ||
        hipMalloc(&s->d_gj_one, 2 * sizeof(int)) != hipSuccess ||
        hipMalloc(&s->d_gj_xoff, sizeof(long long)) != hipSuccess ||
        hipMalloc(&s->d_gj_P, 2 * 32 * 32 * sizeof(double)) != hipSuccess)
      return fail(ADJ_E_OOM, "Gauss-Jordan tables");
    HIPCHK(hipMemcpy(s->d_gj_tiles, tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->d_gj_one, one, 2 * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->d_gj_xoff, &zero, sizeof(long long), hipMemcpyHostToDevice));
    s->gj_mp = mp;
  }
  {
    // block Gauss-Jordan; the pivot block of step k + 1 is formed and
    // inverted beside the tiles of step k (two pivot slots)
    ProfScope p(s, 7, st);
    launch_gj_pad(st, m, mp, s->d_C);
    double* A = s->d_C;
    double* B = s->d_colbuf;
    const int ntiles = (mp / 64) * (mp / 64), nsteps = mp / 32;
    launchb_gj_pivot(st, 1, s->d_gj_one, s->d_gj_xoff, s->d_gj_one + 1, A, s->d_gj_P, s->d_err);
    for (int k = 0; k < nsteps; ++k) {
      ProfScope pk(s, 10, st);
      const bool next = k + 1 < nsteps;
      launchb_gj_step(st, next ? 1 : 0, next ? s->d_gj_one : nullptr, ntiles, s->d_gj_tiles, 32 * k, s->d_gj_xoff,
                      s->d_gj_one + 1, A, B, s->d_gj_P + (k % 2) * 1024, s->d_gj_P + ((k + 1) % 2) * 1024, s->d_err);
      std::swap(A, B);
    }
    s->d_X = A;
  }
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
  std::vector<int> vid(nc), fric(nc);
  if (nc) {
    HIPCHK(hipMemcpyAsync(vid.data(), cst->vid, nc * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(fric.data(), cst->fric, nc * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  drop_chunk_graphs(s);
  s->mu = cst->mu;
  s->symmetric = true;
  if (cst->mu != 0.0)
    for (int c = 0; c < nc; ++c)
      if (fric[c]) s->symmetric = false;
  s->cur_vid = cst->vid;
  s->cur_frame = cst->frame;
  s->cur_q = q;
  // a1 + a2: per-tet Jacobians, gather assembly of Acal^T; the device error
  // flag (inverted element, singular capacitance pivot) starts clear
  launch_fill_int(st, 1, s->d_err, 0);
  launch_fill_int(st, 1, s->d_err + 2, 0);
  {
    ProfScope p(s, 5, st);
    launch_tet_blocks(st, s->nt, s->d_tets, s->d_Bt, s->d_vol, s->d_lmu, s->d_llam, h2, q, s->d_tetblk,
                      s->d_err, s->material);
  }
  {
    ProfScope p(s, 6, st);
    launch_assemble(st, s->nnzb, s->nt, s->d_slot_ptr, s->d_slot_code, s->d_tetblk, s->d_row_of_slot, s->d_col,
                    s->d_mass, s->d_val);
  }
  // a3: contact blocks folded into the diagonal blocks of Acal^T
  launch_contact_blocks(st, nc, cst->fric, cst->frame, cst->delta, cst->lambda, cst->mu, nullptr, s->hs.eps, h2, 1,
                        s->d_Wt, s->d_Q, s->d_kh, s->d_Kc, s->d_kmu);
  launch_contact_fold(st, nc, cst->vid, s->d_diag_slot, s->d_Wt, s->d_val);
  launch_binding_fold(st, s->nb, s->d_bvid, s->d_bE, h2, s->d_diag_slot, s->d_val);
  // a4: Delassus (cached per contact vertex set), capacitance, its inverse;
  // skipped when the solves will use a comparison preconditioner
  const bool woodbury =
      !opts || opts->precond == ADJ_PRECOND_WOODBURY || opts->precond == ADJ_PRECOND_WOODBURY_NO_Z;
  adj_status a = contact_layout(s, st, nc, vid, fric, opts ? opts->reuse_delassus != 0 : true, woodbury,
                                opts && opts->precond == ADJ_PRECOND_WOODBURY_NO_Z);
  if (a != ADJ_OK) return a;
  if (woodbury && (a = build_capacitance(s, st, cst->mu, 1)) != ADJ_OK) return a;
  s->woodbury_ready = woodbury;
  s->mixed_ready = false;
  // entry-major copy of the assembled matrix for the Krylov products, and
  // with ADJ_MIXED its FP32 rounding read by the inner solve (S and S^T have
  // FP32 copies from scene creation).  The Woodbury factors D, X and Z stay
  // FP64: in the directions of stiff contacts the correction cancels
  // A^{-1} r almost exactly, so their rounding would be amplified by the
  // contact-to-elastic stiffness ratio.
  const bool mixed = opts && (opts->prec == ADJ_MIXED || opts->prec == ADJ_MIXED_PC);
  launch_bsr_soa(st, s->nnzb, s->d_val, s->d_valT, mixed ? s->d_val32 : nullptr);
  s->mixed_ready = mixed;
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
  if (err[2]) return fail(ADJ_E_DEVICE, "a pipelined capacitance substitution waited past its limit");
  return ADJ_OK;
}

// P x -> out (x and out distinct from the scratch vectors t1, u, tvec).
// f32: S and S^T are read from their FP32 copies (vectors, X and Z stay FP64).
// A_s^{-1} = S^T S with S = L^{-1} P, applied either as the two sparse-inverse
// products or as two level-scheduled sweeps with L (s->use_sweeps).
// t = X Hq u: the capacitance solve of the Woodbury correction, with the
// explicit inverse X or with the block-LU factors (cap_lu).
static void cap_apply(adj_scene* s, hipStream_t st, const double* u, const GmresState* state, double* t) {
  if (s->cap_lu && s->tune.lu_pipe && lu_group_blocks() == 4)
    launch_wb_lu_pipe(st, s->m, s->mp, s->d_row_c, s->d_row_i, s->cur_vid, s->d_Q, s->d_X, s->d_lu_P, u, state, t,
                      s->d_lu_y, s->d_lu_A0, s->d_lu_A1, s->d_lu_tick, s->d_err);
  else if (s->cap_lu)
    launch_wb_lu(st, s->m, s->mp, s->d_row_c, s->d_row_i, s->cur_vid, s->d_Q, s->d_X, s->d_lu_P, lu_group_blocks(), u,
                 state, t, s->d_lu_y);
  else
    launch_wb_gather(st, s->m, s->mp, s->d_row_c, s->d_row_i, s->cur_vid, s->d_Q, s->d_X, u, state, t);
}

// s_forward: y = S x (x vertex-indexed, the current basis vector scaled when
// state and scale are given; y in elimination order).
static void s_forward(adj_scene* s, hipStream_t st, const double* x, long long stride, const double* scale,
                      const GmresState* state, double* y, bool f32) {
  if (!s->use_sweeps) {
    if (f32)
      launch_spmv_tasks(st, s->nS_tasks, (const int4*)s->d_Stasks, s->d_Sp, s->d_Sj, s->d_Sx32, x, stride, scale,
                        state, y);
    else
      launch_spmv_tasks(st, s->nS_tasks, (const int4*)s->d_Stasks, s->d_Sp, s->d_Sj, s->d_Sx, x, stride, scale,
                        state, y);
    return;
  }
  const HostScene& h = s->hs;
  launch_perm_gather(st, s->nv, s->d_perm, x, stride, scale, state, s->d_lt);
  if (s->fuse_k > 0) {
    if (f32)
      launch_sweep_parts(st, s->n_parts, 1, s->fuse_k, s->d_part_rows, s->d_part_off, s->d_Fp, s->d_Fj, s->d_Fx32,
                         s->d_Ip, s->d_Ij, s->d_Ix32, state, y, s->d_lt);
    else
      launch_sweep_parts(st, s->n_parts, 1, s->fuse_k, s->d_part_rows, s->d_part_off, s->d_Fp, s->d_Fj, s->d_Fx,
                         s->d_Ip, s->d_Ij, s->d_Ix, state, y, s->d_lt);
  }
  for (int l = s->fuse_k; l < s->n_levels; ++l) {
    const int a0 = h.fA_off[l], na = h.fA_off[l + 1] - a0, b0 = h.fB_off[l], nb = h.fB_off[l + 1] - b0;
    const int4* ta = (const int4*)s->d_fA + a0;
    const int4* tb = (const int4*)s->d_fB + b0;
    if (f32) {
      launch_spmv_tasks_acc(st, na, ta, s->d_Fp, s->d_Fj, s->d_Fx32, y, -1.0, state, s->d_lt);
      if (nb) launch_spmv_tasks(st, nb, tb, s->d_Ip, s->d_Ij, s->d_Ix32, s->d_lt, 0, nullptr, state, y);
    } else {
      launch_spmv_tasks_acc(st, na, ta, s->d_Fp, s->d_Fj, s->d_Fx, y, -1.0, state, s->d_lt);
      if (nb) launch_spmv_tasks(st, nb, tb, s->d_Ip, s->d_Ij, s->d_Ix, s->d_lt, 0, nullptr, state, y);
    }
  }
}

// s_transpose: out = S^T y (y in elimination order, out vertex-indexed).
static void s_transpose(adj_scene* s, hipStream_t st, const double* y, const GmresState* state, double* out,
                        bool f32) {
  if (!s->use_sweeps) {
    if (f32)
      launch_spmv_tasks(st, s->nST_tasks, (const int4*)s->d_STtasks, s->d_STp, s->d_STj, s->d_STx32, y, 0, nullptr,
                        state, out);
    else
      launch_spmv_tasks(st, s->nST_tasks, (const int4*)s->d_STtasks, s->d_STp, s->d_STj, s->d_STx, y, 0, nullptr,
                        state, out);
    return;
  }
  const HostScene& h = s->hs;
  (void)hipMemcpyAsync(s->d_lt, y, (size_t)s->n3 * sizeof(double), hipMemcpyDeviceToDevice, st);
  for (int l = s->n_levels - 1; l >= s->fuse_k; --l) {
    const int a0 = h.bA_off[l], na = h.bA_off[l + 1] - a0, b0 = h.bB_off[l], nb = h.bB_off[l + 1] - b0;
    const int4* ta = (const int4*)s->d_bA + a0;
    const int4* tb = (const int4*)s->d_bB + b0;
    if (f32) {
      launch_spmv_tasks_acc(st, na, ta, s->d_Bp, s->d_Bj, s->d_Bx32, s->d_lz, -1.0, state, s->d_lt);
      if (nb) launch_spmv_tasks(st, nb, tb, s->d_ITp, s->d_ITj, s->d_ITx32, s->d_lt, 0, nullptr, state, s->d_lz);
    } else {
      launch_spmv_tasks_acc(st, na, ta, s->d_Bp, s->d_Bj, s->d_Bx, s->d_lz, -1.0, state, s->d_lt);
      if (nb) launch_spmv_tasks(st, nb, tb, s->d_ITp, s->d_ITj, s->d_ITx, s->d_lt, 0, nullptr, state, s->d_lz);
    }
  }
  if (s->fuse_k > 0) {
    if (f32)
      launch_sweep_parts(st, s->n_parts, 0, s->fuse_k, s->d_part_rows, s->d_part_off, s->d_Bp, s->d_Bj, s->d_Bx32,
                         s->d_ITp, s->d_ITj, s->d_ITx32, state, s->d_lz, s->d_lt);
    else
      launch_sweep_parts(st, s->n_parts, 0, s->fuse_k, s->d_part_rows, s->d_part_off, s->d_Bp, s->d_Bj, s->d_Bx,
                         s->d_ITp, s->d_ITj, s->d_ITx, state, s->d_lz, s->d_lt);
  }
  launch_perm_scatter(st, s->nv, s->d_perm, s->d_lz, state, out);
}

// Sweeps or products: tune.a_inv 2 / 1, or automatically sweeps when S holds
// far more entries than L (large scenes, where the products are bound by
// streaming S) and the products otherwise (small scenes, where the sweeps'
// level launches would dominate).
static void choose_a_inv(adj_scene* s) {
  const long long nnzL = (long long)s->hs.Li.size();
  const bool big = s->nnzS >= 32000000LL && s->nnzS >= 4 * nnzL;
  const bool want = s->tune.a_inv == 2 || (s->tune.a_inv == 0 && big);
  if (want && s->sweeps_built) {
    if (!s->use_sweeps) drop_chunk_graphs(s);
    s->use_sweeps = true;
  } else {
    if (s->use_sweeps) drop_chunk_graphs(s);
    s->use_sweeps = false;
  }
}

static void apply_precond(adj_scene* s, hipStream_t st, const double* x, long long stride,
                          const double* scale, const GmresState* state, double* out, bool f32 = false) {
  const double h2 = s->hs.h * s->hs.h;
  if (s->precond == ADJ_PRECOND_JACOBI || s->precond == ADJ_PRECOND_POINT_JACOBI) {
    const int point = s->precond == ADJ_PRECOND_POINT_JACOBI ? 1 : 0;
    // the diagonal blocks are read in FP64 in both modes (they hold the stiff contact terms)
    launch_block_jacobi(st, s->nv, s->d_diag_slot, s->d_val, x, stride, scale, state, point, out);
    return;
  }
  const bool woodbury =
      s->nc > 0 && (s->precond == ADJ_PRECOND_WOODBURY || s->precond == ADJ_PRECOND_WOODBURY_NO_Z);
  {
    ProfScope p(s, 0, st);
    s_forward(s, st, x, stride, scale, state, s->d_t1, f32);
  }
  if (woodbury && !s->use_z) {
    // Correction through Y = S E:  A^{-1} r - h^2 A^{-1} H^T t' =
    // S^T (S r - h^2 Y H^T t'), with t' = X H A^{-1} r and H A^{-1} r the
    // contact-vertex rows of S^T (S r) (= Y^T S r).  One S and one S^T
    // product per apply; Y and the contact rows are FP64 in both modes, so
    // that H out = (I - h^2 Y^T Y X) H A^{-1} r holds with the same Y as the
    // Delassus matrix D = Y^T Y of X: for stiff contacts the correction
    // cancels A^{-1} r almost exactly in the contact directions, and any
    // inconsistency there would be amplified by the contact-to-elastic
    // stiffness ratio.  With FP32 products the contact rows of the result
    // are therefore recomputed in FP64 from the same S r.
    launch_spmv_tasks(st, s->nCT_tasks, (const int4*)s->d_CTtasks, s->d_STp, s->d_STj, s->d_STx, s->d_t1, 0, nullptr,
                      state, s->d_u);
    {
      ProfScope p(s, 2, st);
      cap_apply(s, st, s->d_u, state, s->d_tvec);
    }
    ProfScope p(s, 3, st);
    launch_fill_zero(st, (size_t)s->n3, s->d_wz);
    launch_scatter_ht(st, s->ncv, s->d_cv, s->d_cv_ptr, s->d_c_row0, s->d_c_nrow, s->d_Q, s->d_tvec, state, s->d_wz);
    launch_spmv_tasks_acc(st, s->nY_tasks, (const int4*)s->d_Ytasks, s->d_Yp, s->d_Ycol, s->d_Yval, s->d_wz, -h2,
                          state, s->d_t1);
    {
      ProfScope p1(s, 1, st);
      s_transpose(s, st, s->d_t1, state, out, f32);
    }
    if (f32)
      launch_spmv_tasks(st, s->nCT_tasks, (const int4*)s->d_CTtasks, s->d_STp, s->d_STj, s->d_STx, s->d_t1, 0,
                        nullptr, state, out);
    return;
  }
  double* u = woodbury ? s->d_u : out;
  {
    ProfScope p(s, 1, st);
    s_transpose(s, st, s->d_t1, state, u, f32);
  }
  if (!woodbury) return;
  {
    ProfScope p(s, 2, st);
    cap_apply(s, st, s->d_u, state, s->d_tvec);
  }
  ProfScope p(s, 3, st);
  if (s->use_z) {
    launch_wb_correct(st, s->nv, s->ncv, s->d_cv_ptr, s->d_c_row0, s->d_c_nrow, s->d_Q, s->d_tvec, s->d_Z, h2,
                      s->d_u, state, out);
    return;
  }
}

static void bsr(adj_scene* s, hipStream_t st, const double* x, double* outbase, long long stride,
                const GmresState* state, bool f32) {
  if (f32)
    launch_bsr_spmv(st, s->tune.bsr_lanes, s->nv, s->d_rowptr, s->d_col, s->d_val32, s->d_valT, s->nnzb, x, outbase, stride,
                    state);
  else
    launch_bsr_spmv(st, s->tune.bsr_lanes, s->nv, s->d_rowptr, s->d_col, s->d_valT, s->nnzb, x, outbase, stride, state);
}

// One GMRES iteration per pass of the loop: preconditioner (4 launches),
// block-sparse product fused with the first Gram-Schmidt dots, the two
// Gram-Schmidt updates (classical Gram-Schmidt applied twice) and the
// one-block Givens step.
// f32: FP32 block values in the product; pc32: FP32 preconditioner.
static void gmres_chunk(adj_scene* s, hipStream_t st, bool f32, bool pc32, int n) {
  const long long n3 = s->n3, stride = n3;
  // above kFoldAt partial blocks the Gram-Schmidt dots are folded once by a
  // separate launch instead of re-added by every block of the next kernel
  constexpr int kFoldAt = 256;
  const int nb1_raw = bsr_blocks(s->nv, s->tune.bsr_lanes), nb2_raw = gm_blocks(n3, s->tune.gs_rows);
  const int nb1 = nb1_raw > kFoldAt ? 1 : nb1_raw, nb2 = nb2_raw > kFoldAt ? 1 : nb2_raw;
  for (int k = 0; k < n; ++k) {
    apply_precond(s, st, s->d_Vt, stride, s->d_scale, s->d_state, s->d_y, pc32);
    {
      ProfScope p(s, 4, st);
      if (f32)
        launch_bsr_dots(st, s->tune.bsr_lanes, s->nv, s->d_rowptr, s->d_col, s->d_val32, s->d_valT, s->nnzb, s->d_y, s->d_Vt, stride,
                        s->d_state, -1, s->P1(), s->d_Zk);
      else
        launch_bsr_dots(st, s->tune.bsr_lanes, s->nv, s->d_rowptr, s->d_col, s->d_valT, s->nnzb, s->d_y, s->d_Vt, stride,
                        s->d_state, -1, s->P1(), s->d_Zk);
    }
    if (nb1_raw > kFoldAt) launch_fold_partials(st, s->P1(), nb1_raw, s->d_state, 0);
    {
      ProfScope p(s, 9, st);
      launch_gm_update(st, n3, s->tune.gs_rows, s->d_Vt, stride, s->d_scale, s->d_state, s->P1(), nb1, s->P2(),
                       s->d_hbuf, 0);
    }
    if (nb2_raw > kFoldAt) launch_fold_partials(st, s->P2(), nb2_raw, s->d_state, 0);
    {
      ProfScope p(s, 8, st);
      launch_gm_update(st, n3, s->tune.gs_rows, s->d_Vt, stride, s->d_scale, s->d_state, s->P2(), nb2, s->P3(),
                       s->d_hbuf, 1);
      launch_gm_givens(st, s->d_state, s->P3(), nb2_raw, s->d_scale, s->d_hbuf, s->d_H, s->d_cs, s->d_sn, s->d_g);
    }
  }
}

// One PCG iteration per pass (see the kernel file for the sequence); p and w
// are basis slots 0 and 1, so the fused product-and-dot kernel gives p . w.
static void pcg_chunk(adj_scene* s, hipStream_t st, bool f32) {
  const long long n3 = s->n3;
  double* p = s->d_Vt;
  double* w = s->d_Vt + n3;
  double* z = s->d_y;
  const int nb1 = bsr_blocks(s->nv, s->tune.bsr_lanes), nbv = vec_blocks(n3);
  for (int k = 0; k < s->tune.chunk; ++k) {
    {
      ProfScope pr(s, 4, st);
      if (f32)
        launch_bsr_dots(st, s->tune.bsr_lanes, s->nv, s->d_rowptr, s->d_col, s->d_val32, s->d_valT, s->nnzb, p, s->d_Vt, n3,
                        s->d_state, 0, s->P1());
      else
        launch_bsr_dots(st, s->tune.bsr_lanes, s->nv, s->d_rowptr, s->d_col, s->d_valT, s->nnzb, p, s->d_Vt, n3,
                        s->d_state, 0, s->P1());
    }
    launch_pcg_xr(st, n3, s->d_x_pcg, s->d_r, p, w, s->P1(), nb1, s->d_state, s->d_coef, s->P3());
    apply_precond(s, st, s->d_r, 0, nullptr, s->d_state, z, f32);
    launch_dot_partials(st, n3, s->d_r, z, s->d_state, s->P2());
    launch_pcg_scalar(st, s->d_state, s->P2(), nbv, s->P3(), nbv, s->P1(), nb1, s->d_coef, 0);
    launch_pcg_p(st, n3, z, p, s->d_state, s->d_coef);
  }
}

// One chunk of Krylov iterations (kind 0 GMRES, 1 PCG) on `st`: launched
// directly (n GMRES iterations), or (tuning.graph = 1, no live profiling)
// replayed from a graph of tuning.chunk iterations captured on the scene's
// private stream after the last setup.
static hipError_t run_chunk(adj_scene* s, hipStream_t st, int kind, bool f32, int n, bool pc32) {
  if (!s->tune.graph || s->prof_kernel >= 0) {
    if (kind == 0)
      gmres_chunk(s, st, f32, pc32, n);
    else
      pcg_chunk(s, st, f32);
    return hipGetLastError();
  }
  hipGraphExec_t& ex = s->chunk_exec[4 * kind + (pc32 ? 2 : 0) + (f32 ? 1 : 0)];
  if (!ex) {
    hipError_t e;
    if (!s->cap_stream && (e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking)) != hipSuccess)
      return e;
    if ((e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    if (kind == 0)
      gmres_chunk(s, s->cap_stream, f32, pc32, s->tune.chunk);
    else
      pcg_chunk(s, s->cap_stream, f32);
    hipGraph_t g = nullptr;
    if ((e = hipStreamEndCapture(s->cap_stream, &g)) != hipSuccess) return e;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      ex = nullptr;
      return e;
    }
  }
  return hipGraphLaunch(ex, st);
}

// Right-preconditioned restarted GMRES on the assembled matrix (s->d_val,
// contacts folded) with the current Woodbury preconditioner: x = A^{-1} b.
static adj_status gmres_solve(adj_scene* s, hipStream_t st, const double* b, double* x, double rtol,
                              int maxit, int R, int* iters_out, double* relres_out, bool* converged_out,
                              bool f32 = false, bool verify = true, bool pc32 = false) {
  pc32 = pc32 || f32;
  const long long n3 = s->n3;
  const long long stride = n3;
  if (b != s->d_b) HIPCHK(hipMemcpyAsync(s->d_b, b, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  launch_fill_zero(st, (size_t)n3, x);
  launch_fill_zero(st, (size_t)n3, s->d_r);
  GmresState init{};
  init.restart = R;
  init.tol = 0.0;
  HIPCHK(hipMemcpyAsync(s->d_state, &init, sizeof(GmresState), hipMemcpyHostToDevice, st));
  launch_residual(st, n3, s->d_b, s->d_r, s->d_Vt, s->P3(), s->d_state, s->d_scale,
                  s->d_g);
  HIPCHK(hipMemcpyAsync(s->h_state, s->d_state, sizeof(GmresState), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double bnorm = s->h_state->rnorm;
  const double tol = rtol * bnorm;
  if (!std::isfinite(bnorm)) return fail(ADJ_E_ARG, "non-finite right-hand side");
  GmresState cur = *s->h_state;
  cur.tol = tol;
  cur.restart = R;
  cur.active = (bnorm > tol) ? 1 : 0;
  HIPCHK(hipMemcpyAsync(s->d_state, &cur, sizeof(GmresState), hipMemcpyHostToDevice, st));
  int total = 0;
  double relres = (bnorm > 0) ? cur.rnorm / bnorm : 0.0;
  bool converged = !(bnorm > tol);
  // Iterations per chunk: tuning.chunk at first, then the number the mean
  // residual reduction per iteration so far predicts to reach tol (at least
  // one), so that few iterations past convergence are enqueued (each costs
  // its launches even when the state mask makes its kernels return early).
  double rate = 0.0;
  auto predicted = [&](double res) {
    if (!(rate > 0.0 && rate < 1.0) || !(res > tol)) return s->tune.chunk;
    const double need = std::ceil(std::log(tol / res) / std::log(rate));
    return (int)std::max(1.0, std::min((double)s->tune.chunk, need));
  };
  double r_cycle = cur.rnorm;
  while (!converged && total < maxit) {
    int done_in_cycle = 0;
    int n = predicted(r_cycle);
    double r_prev = r_cycle;
    int j_prev = 0;
    while (true) {
      HIPCHK(run_chunk(s, st, 0, f32, n, pc32));
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(s->h_state, s->d_state, sizeof(GmresState), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      done_in_cycle = s->h_state->j;
      if (!s->h_state->active || total + done_in_cycle >= maxit) break;
      const double res = s->h_state->res;
      if (done_in_cycle > j_prev && res > 0.0 && res < r_prev)
        rate = std::pow(res / r_prev, 1.0 / (done_in_cycle - j_prev));
      r_prev = res;
      j_prev = done_in_cycle;
      n = predicted(res);
    }
    total += done_in_cycle;
    // flexible GMRES: x += Zk y with the stored preconditioned vectors
    // Zk_j = M^-1 v_j (no further preconditioner application)
    launch_gm_finish(st, n3, s->d_state, s->d_H, s->d_g, nullptr, s->d_Zk, stride, s->d_coef, s->d_dz);
    launch_axpy(st, n3, 1.0, s->d_dz, x);
    if (!verify && s->h_state->res <= tol) {
      // an inner solve of the refinement: the caller forms the true
      // residual itself, so the recurrence's estimate ends the solve
      relres = (bnorm > 0) ? s->h_state->res / bnorm : 0.0;
      converged = true;
      break;
    }
    bsr(s, st, x, s->d_r, 0, nullptr, f32);
    launch_residual(st, n3, s->d_b, s->d_r, s->d_Vt, s->P3(), s->d_state, s->d_scale,
                    s->d_g);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(s->h_state, s->d_state, sizeof(GmresState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    relres = (bnorm > 0) ? s->h_state->rnorm / bnorm : 0.0;
    if (!std::isfinite(relres)) return fail(ADJ_E_SINGULAR, "non-finite residual in the Krylov solve");
    converged = s->h_state->rnorm <= tol;
    r_cycle = s->h_state->rnorm;
    if (done_in_cycle == 0 && !converged) break;  // no progress possible
  }
  *iters_out = total;
  *relres_out = relres;
  *converged_out = converged;
  return ADJ_OK;
}

// Preconditioned conjugate gradients (symmetric case), same preconditioner
// and stopping rule as GMRES; the recurrence residual is confirmed by the
// true residual, and the iteration restarts from the current x if they
// disagree.  p = Vt_0, w = Vt_1, z = y; device scalars in coef[0..3].
static adj_status pcg_solve(adj_scene* s, hipStream_t st, const double* b, double* x, double rtol, int maxit,
                            int* iters_out, double* relres_out, bool* converged_out, bool f32 = false) {
  const long long n3 = s->n3;
  double* p = s->d_Vt;
  double* z = s->d_y;
  double* xi = s->d_x_pcg;  // fixed address, so a captured chunk stays valid
  double* sc = s->d_coef;
  if (b != s->d_b) HIPCHK(hipMemcpyAsync(s->d_b, b, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  launch_fill_zero(st, (size_t)n3, xi);
  launch_fill_zero(st, (size_t)n3, s->d_r);
  GmresState init{};
  HIPCHK(hipMemcpyAsync(s->d_state, &init, sizeof(GmresState), hipMemcpyHostToDevice, st));
  launch_residual(st, n3, s->d_b, s->d_r, nullptr, s->P3(), s->d_state, nullptr, nullptr);
  HIPCHK(hipMemcpyAsync(s->h_state, s->d_state, sizeof(GmresState), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double bnorm = s->h_state->rnorm;
  const double tol = rtol * bnorm;
  if (!std::isfinite(bnorm)) return fail(ADJ_E_ARG, "non-finite right-hand side");
  double rnorm = bnorm;
  int total = 0;
  bool converged = !(bnorm > tol);
  for (int pass = 0; pass < 8 && !converged && total < maxit; ++pass) {
    GmresState cur{};
    cur.tol = tol;
    cur.restart = maxit - total;
    cur.res = rnorm;
    cur.rnorm = rnorm;
    cur.active = 1;
    HIPCHK(hipMemcpyAsync(s->d_state, &cur, sizeof(GmresState), hipMemcpyHostToDevice, st));
    apply_precond(s, st, s->d_r, 0, nullptr, s->d_state, z, f32);
    launch_dot_partials(st, n3, s->d_r, z, s->d_state, s->P2());
    launch_pcg_scalar(st, s->d_state, s->P2(), vec_blocks(n3), nullptr, 0, nullptr, 0, sc, 1);
    launch_fill_zero(st, (size_t)n3, p);
    launch_pcg_p(st, n3, z, p, s->d_state, sc);
    int done = 0;
    while (true) {
      HIPCHK(run_chunk(s, st, 1, f32, s->tune.chunk, f32));
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(s->h_state, s->d_state, sizeof(GmresState), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      done = s->h_state->j;
      if (!s->h_state->active) break;
    }
    total += done;
    // true residual
    bsr(s, st, xi, s->d_r, 0, nullptr, f32);
    launch_residual(st, n3, s->d_b, s->d_r, nullptr, s->P3(), s->d_state, nullptr, nullptr);
    HIPCHK(hipMemcpyAsync(s->h_state, s->d_state, sizeof(GmresState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rnorm = s->h_state->rnorm;
    if (!std::isfinite(rnorm)) return fail(ADJ_E_SINGULAR, "non-finite residual in the Krylov solve");
    converged = rnorm <= tol;
    if (done == 0) break;  // breakdown without progress
  }
  HIPCHK(hipMemcpyAsync(x, xi, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  *iters_out = total;
  *relres_out = (bnorm > 0) ? rnorm / bnorm : 0.0;
  *converged_out = converged;
  return ADJ_OK;
}

// Semi-implicit fixed-point iteration x <- x + A^{-1} (b - Acal^T x)
// (A^{-1} = S^T S), FP64; the residual is checked every 16 sweeps; stops at
// the tolerance, at maxit, or when the residual exceeds 1e6 |b| (diverged).
static adj_status semi_implicit_solve(adj_scene* s, hipStream_t st, const double* b, double* x, double rtol,
                                      int maxit, int* iters, double* relres, bool* conv) {
  const long long n3 = s->n3;
  launch_fill_zero(st, (size_t)n3, x);
  auto residual = [&]() {  // d_r = b - Acal^T x
    bsr(s, st, x, s->d_r, 0, nullptr, false);
    launch_axpy(st, n3, -1.0, b, s->d_r);
    launch_scale_vec(st, n3, s->d_r, -1.0, s->d_r);
  };
  double nb[2];
  launch_norms(st, n3, b, s->P3(), s->d_norms);
  HIPCHK(hipMemcpyAsync(nb, s->d_norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double bnorm = std::sqrt(nb[0]);
  double rn = bnorm;
  if (!std::isfinite(bnorm)) return fail(ADJ_E_ARG, "non-finite right-hand side");
  int it = 0;
  while (it < maxit && rn > rtol * bnorm) {
    const int chunk = std::min(16, maxit - it);
    for (int k = 0; k < chunk; ++k) {
      residual();
      launch_spmv_tasks(st, s->nS_tasks, (const int4*)s->d_Stasks, s->d_Sp, s->d_Sj, s->d_Sx, s->d_r, 0, nullptr,
                        nullptr, s->d_t1);
      launch_spmv_tasks(st, s->nST_tasks, (const int4*)s->d_STtasks, s->d_STp, s->d_STj, s->d_STx, s->d_t1, 0,
                        nullptr, nullptr, s->d_dz);
      launch_axpy(st, n3, 1.0, s->d_dz, x);
    }
    it += chunk;
    residual();
    launch_norms(st, n3, s->d_r, s->P3(), s->d_norms);
    HIPCHK(hipMemcpyAsync(nb, s->d_norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rn = std::sqrt(nb[0]);
    if (!std::isfinite(rn) || rn > 1e6 * bnorm) break;  // diverged
  }
  *iters = it;
  *relres = bnorm > 0 ? rn / bnorm : 0.0;
  *conv = rn <= rtol * bnorm;
  return ADJ_OK;
}

static adj_status krylov_solve(adj_scene* s, hipStream_t st, bool use_pcg, const double* b, double* x,
                               double rtol, int maxit, int R, int* iters, double* relres, bool* conv, bool f32,
                               bool verify = true) {
  if (use_pcg) return pcg_solve(s, st, b, x, rtol, maxit, iters, relres, conv, f32);
  return gmres_solve(s, st, b, x, rtol, maxit, R, iters, relres, conv, f32, verify);
}

static adj_status adjoint_solve_impl(adj_scene* s, const double* dL_dq, const double* dL_dv, double* z,
                                     const adj_solve_opts* opts, adj_solve_info* info, void* stream);

// The device error flag raised by the last setup (inverted element,
// singular capacitance pivot) takes precedence over the solve's own status.
extern "C" adj_status adjoint_solve(adj_scene* s, const double* dL_dq, const double* dL_dv, double* z,
                                    const adj_solve_opts* opts, adj_solve_info* info, void* stream) {
  const adj_status a = adjoint_solve_impl(s, dL_dq, dL_dv, z, opts, info, stream);
  if (a == ADJ_E_ARG || a == ADJ_E_SHAPE || a == ADJ_E_NOTIMPL) return a;
  const adj_status e = adj_check_status(s, stream);
  return e != ADJ_OK ? e : a;
}

static adj_status adjoint_solve_impl(adj_scene* s, const double* dL_dq, const double* dL_dv, double* z,
                                     const adj_solve_opts* opts, adj_solve_info* info, void* stream) {
  if (!s || !dL_dq || !dL_dv || !z || !opts) return fail(ADJ_E_ARG, "null argument");
  if (!s->setup_done) return fail(ADJ_E_ARG, "adjoint_setup has not run");
  if (!(opts->rtol > 0) || opts->maxit <= 0 || opts->restart < 1 || opts->restart > kMaxRestart)
    return fail(ADJ_E_ARG, "invalid solve options");
  if (opts->prec != ADJ_FP64 && opts->prec != ADJ_MIXED && opts->prec != ADJ_MIXED_PC)
    return fail(ADJ_E_ARG, "unknown precision");
  if (opts->method != ADJ_AUTO && opts->method != ADJ_GMRES && opts->method != ADJ_PCG &&
      opts->method != ADJ_SEMI_IMPLICIT)
    return fail(ADJ_E_ARG, "unknown Krylov method");
  if (opts->method == ADJ_SEMI_IMPLICIT && opts->prec != ADJ_FP64)
    return fail(ADJ_E_NOTIMPL, "the semi-implicit iteration runs in FP64");
  if (opts->precond != ADJ_PRECOND_WOODBURY && opts->precond != ADJ_PRECOND_SPARSE_INVERSE &&
      opts->precond != ADJ_PRECOND_JACOBI && opts->precond != ADJ_PRECOND_POINT_JACOBI &&
      opts->precond != ADJ_PRECOND_WOODBURY_NO_Z)
    return fail(ADJ_E_ARG, "unknown preconditioner");
  if ((opts->precond == ADJ_PRECOND_WOODBURY || opts->precond == ADJ_PRECOND_WOODBURY_NO_Z) && s->nc > 0 &&
      !s->woodbury_ready)
    return fail(ADJ_E_ARG, "the last adjoint_setup skipped the Woodbury factors (it ran with another precond)");
  if (opts->precond != s->precond) {
    drop_chunk_graphs(s);  // captured chunks hold the preconditioner's launches
    s->precond = opts->precond;
  }
  if (opts->method == ADJ_PCG && !s->symmetric)
    return fail(ADJ_E_ARG, "PCG needs a symmetric system (no frictional contact, or mu = 0)");
  const bool use_pcg = opts->method == ADJ_PCG || (opts->method == ADJ_AUTO && s->symmetric);
  if (opts->prec != ADJ_FP64 && !s->mixed_ready)
    return fail(ADJ_E_ARG, "adjoint_setup must run with ADJ_MIXED or ADJ_MIXED_PC before a mixed solve");
  hipStream_t st = (hipStream_t)stream;
  const long long n3 = s->n3;
  choose_a_inv(s);
  // b = dL_dq + dL_dv / h
  HIPCHK(hipMemcpyAsync(s->d_rhs, dL_dq, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  launch_axpy(st, n3, 1.0 / s->hs.h, dL_dv, s->d_rhs);
  int total = 0, refine = 0;
  double relres = 0.0;
  bool converged = false;
  adj_status a;
  if (opts->method == ADJ_SEMI_IMPLICIT) {
    a = semi_implicit_solve(s, st, s->d_rhs, z, opts->rtol, opts->maxit, &total, &relres, &converged);
    if (a != ADJ_OK) return a;
  } else if (opts->prec == ADJ_FP64 && !(opts->max_refine > 0 && opts->rtol < kFp64Floor)) {
    a = krylov_solve(s, st, use_pcg, s->d_rhs, z, opts->rtol, opts->maxit, opts->restart, &total, &relres,
                     &converged, false);
    if (a != ADJ_OK) return a;
  } else if (opts->prec == ADJ_MIXED_PC && !use_pcg) {
    // FP32 preconditioner inside FP64 flexible GMRES: the product, the
    // Gram-Schmidt and the residual recurrence stay FP64, and the solution
    // is formed from the stored preconditioned vectors, so the rounding of
    // the FP32 sparse inverse (or sweeps) changes the iterates, not the
    // residual that ends the solve (no refinement passes).
    a = gmres_solve(s, st, s->d_rhs, z, opts->rtol, opts->maxit, opts->restart, &total, &relres, &converged, false,
                    true, true);
    if (a != ADJ_OK) return a;
  } else {
    // Iterative refinement.  Mixed: FP64 residual r = b - Acal^T z with the
    // FP64 matrix, inner GMRES with FP32-stored matrices on Acal^T dz = r.
    // FP64 below the FP64 Krylov floor (rtol < kFp64Floor with max_refine >
    // 0): inner FP64 solves to the floor, residual in double-double.
    const bool f32 = opts->prec != ADJ_FP64;  // ADJ_MIXED_PC with PCG: as ADJ_MIXED
    const double floor_inner = f32 ? 1e-6 : kFp64Floor;
    launch_fill_zero(st, (size_t)n3, z);
    HIPCHK(hipMemcpyAsync(s->d_fu, s->d_rhs, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_norms(st, n3, s->d_rhs, s->P3(), s->d_norms);
    double nb[2];
    HIPCHK(hipMemcpyAsync(nb, s->d_norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double bnorm = std::sqrt(nb[0]);
    double rnorm = bnorm;
    if (!std::isfinite(bnorm)) return fail(ADJ_E_ARG, "non-finite right-hand side");
    relres = bnorm > 0 ? 1.0 : 0.0;
    converged = !(bnorm > 0);
    for (refine = 0; refine <= std::max(0, opts->max_refine) && !converged && total < opts->maxit; ++refine) {
      const double inner = std::max(floor_inner, 0.5 * opts->rtol * bnorm / rnorm);
      int it = 0;
      double rr = 0.0;
      bool cv = false;
      if ((a = krylov_solve(s, st, use_pcg, s->d_fu, s->d_du, inner, opts->maxit - total, opts->restart, &it,
                            &rr, &cv, f32, false)) != ADJ_OK)
        return a;
      total += it;
      const double r_before = rnorm;
      auto residual = [&]() -> adj_status {
        // r = b - Acal^T z with the FP64 matrix (double-double sums below the FP64 floor)
        if (f32) {
          bsr(s, st, z, s->d_fu, 0, nullptr, false);
          launch_add_vec(st, n3, s->d_rhs, s->d_fu, -1.0, s->d_fu);
        } else {
          launch_bsr_residual_dd(st, s->nv, s->d_rowptr, s->d_col, s->d_val, z, s->d_rhs, s->d_fu);
        }
        launch_norms(st, n3, s->d_fu, s->P3(), s->d_norms);
        HIPCHK(hipMemcpyAsync(nb, s->d_norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        rnorm = std::sqrt(nb[0]);
        relres = rnorm / bnorm;
        return ADJ_OK;
      };
      launch_axpy(st, n3, 1.0, s->d_du, z);
      if ((a = residual()) != ADJ_OK) return a;
      if (!f32 && !(rnorm < r_before)) {
        launch_axpy(st, n3, -1.0, s->d_du, z);  // no further progress in FP64: keep the better iterate
        if ((a = residual()) != ADJ_OK) return a;
        converged = relres <= opts->rtol;
        break;
      }
      if (!(rnorm < r_before)) {
        // The FP32 inner solve did not reduce the residual (contacts so stiff
        // that FP32 rounding of A^{-1} r is amplified past the correction):
        // undo the pass and finish in FP64 from the last good iterate.
        launch_axpy(st, n3, -1.0, s->d_du, z);
        if ((a = residual()) != ADJ_OK) return a;
        s->mixed_fallbacks++;
        int it2 = 0;
        double rr2 = 0.0;
        bool cv2 = false;
        if ((a = krylov_solve(s, st, use_pcg, s->d_fu, s->d_du, std::min(1.0, opts->rtol * bnorm / rnorm),
                              std::max(1, opts->maxit - total), opts->restart, &it2, &rr2, &cv2, false)) != ADJ_OK)
          return a;
        total += it2;
        launch_axpy(st, n3, 1.0, s->d_du, z);
        if ((a = residual()) != ADJ_OK) return a;
        ++refine;
        converged = relres <= opts->rtol;
        break;
      }
      if (!std::isfinite(relres)) return fail(ADJ_E_SINGULAR, "non-finite residual in the refinement");
      converged = relres <= opts->rtol;
    }
  }
  if (info) {
    info->iters = total;
    info->refine_steps = refine;
    info->n_contacts = s->nc;
    info->m_rows = s->m;
    info->relres = relres;
    info->delassus_rebuilt = s->delassus_rebuilt;
    info->method = opts->method == ADJ_SEMI_IMPLICIT ? ADJ_SEMI_IMPLICIT : (use_pcg ? ADJ_PCG : ADJ_GMRES);
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
                      s->P1(), grad3, nullptr);
  launch_vjp_tets(st, s->nt, s->d_tets, s->d_Bt, s->d_vol, s->d_lmu, s->d_llam, s->d_E, s->d_nu, h2,
                  s->cur_q, z, dE_tet, dnu_tet, s->P2(), grad3, s->material);
  HIPCHK(hipGetLastError());
  return ADJ_OK;
}

// Allocation-free variant of vjp_params.  Its reductions (per-block partial
// sums of dL/dmu over the contacts and of dL/dE, dL/dnu over the tets) go to
// a fixed file-scope device array instead of the scene's workspace.  On the
// host the array's name only stands for the device symbol: its address on a
// device comes from hipGetSymbolAddress, taken once per device on the first
// call made with that device current, and only that address is handed to
// kernels.  Each device holds its own copy until the process ends; every
// call on a device shares it (no partial needs clearing: each block writes
// its own), so calls that overlap on one device race.
constexpr size_t kScratchDoubles = 65536;  // 512 KiB: up to about 8.3 million tets
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kScratchDevices = 64;
static double* g_scratch_dev[kScratchDevices] = {};
static std::mutex g_scratch_mu;

static adj_status scratch_address(double** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return fail(ADJ_E_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ADJ_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return ADJ_OK;
}

extern "C" adj_status vjp_params_noalloc(adj_scene* s, const double* z, const double* dL_dv, double* dL_dqbar,
                                         double* dL_dvbar, double* dL_dfext, double* grad3, double* dE_tet,
                                         double* dnu_tet, void* stream) {
  if (!s || !z || !dL_dv || !dL_dqbar || !dL_dvbar || !dL_dfext || !grad3)
    return fail(ADJ_E_ARG, "null argument");
  if (!s->setup_done) return fail(ADJ_E_ARG, "adjoint_setup has not run");
  const size_t nbc = ((size_t)s->nc + 255) / 256, nbt = ((size_t)s->nt + 255) / 256;
  if (nbc + 2 * nbt > kScratchDoubles)
    return fail(ADJ_E_SHAPE, "scene too large for the fixed scratch of vjp_params_noalloc (at most " +
                                 std::to_string(kScratchDoubles) + " partial sums: about 8.3 million tets)");
  double* ptr = nullptr;
  adj_status a = scratch_address(&ptr);
  if (a != ADJ_OK) return a;
  hipStream_t st = (hipStream_t)stream;
  const double h = s->hs.h, h2 = h * h;
  launch_vjp_vectors(st, s->nv, z, dL_dv, s->d_mass, h, dL_dqbar, dL_dvbar, dL_dfext);
  launch_vjp_contacts(st, s->nc, s->cur_vid, s->cur_frame, s->d_Kc, s->d_kmu, z, h2, dL_dqbar, ptr, grad3,
                      nullptr);
  launch_vjp_tets(st, s->nt, s->d_tets, s->d_Bt, s->d_vol, s->d_lmu, s->d_llam, s->d_E, s->d_nu, h2, s->cur_q, z,
                  dE_tet, dnu_tet, ptr + nbc, grad3, s->material);
  HIPCHK(hipGetLastError());
  return ADJ_OK;
}

extern "C" adj_status adj_binding_vjp(adj_scene* s, const double* z, const double* q, const double* targets,
                                      double* dL_dtargets, double* dL_dE, void* stream) {
  if (!s || !z || !q) return fail(ADJ_E_ARG, "null argument");
  if (!s->nb) return ADJ_OK;
  if (!targets || !dL_dtargets || !dL_dE) return fail(ADJ_E_ARG, "null binding array");
  const double h2 = s->hs.h * s->hs.h;
  launch_binding_vjp((hipStream_t)stream, s->nb, s->d_bvid, s->d_bE, h2, z, q, targets, dL_dtargets, dL_dE);
  HIPCHK(hipGetLastError());
  return ADJ_OK;
}

static bool valid_tuning(const adj_tuning& t) {
  const bool gs = t.gs_rows == 64 || t.gs_rows == 128 || t.gs_rows == 256;
  const bool ln = t.bsr_lanes == 4 || t.bsr_lanes == 8 || t.bsr_lanes == 16 || t.bsr_lanes == 32;
  const bool gw = t.gj_wide_min >= 128 && t.gj_wide_min % 128 == 0;
  const bool ai = t.a_inv >= 0 && t.a_inv <= 2;
  const bool lu = t.lu_min >= 128 && t.lu_min % 128 == 0 && (t.lu_pipe == 0 || t.lu_pipe == 1) &&
                  t.sweep_fuse >= -1 && t.sweep_fuse <= 64;
  return gs && ln && gw && ai && lu && t.chunk >= 1 && t.chunk <= 64 && (t.graph == 0 || t.graph == 1);
}

extern "C" adj_status adj_set_tuning(adj_scene* s, const adj_tuning* t) {
  if (!s || !t) return fail(ADJ_E_ARG, "null argument");
  if (!valid_tuning(*t)) return fail(ADJ_E_ARG, "tuning value outside the supported set");
  s->tune = *t;
  drop_chunk_graphs(s);
  return prepare_sweep_parts(s);
}

extern "C" adj_status adj_get_tuning(const adj_scene* s, adj_tuning* t) {
  if (!s || !t) return fail(ADJ_E_ARG, "null argument");
  *t = s->tune;
  return ADJ_OK;
}

// Coordinate descent over the launch shapes; each candidate is timed as the
// best of `reps` full solves (HIP events), with captured chunks dropped
// before every solve so that graph replay pays its capture as it would
// after a fresh setup.
extern "C" adj_status adj_autotune(adj_scene* s, const double* dL_dq, const double* dL_dv, double* z,
                                   const adj_solve_opts* opts, int32_t reps, adj_tuning* best, void* stream) {
  if (!s || !dL_dq || !dL_dv || !z || !opts || !best) return fail(ADJ_E_ARG, "null argument");
  if (!s->setup_done) return fail(ADJ_E_ARG, "adjoint_setup has not run");
  if (s->prof_kernel >= 0) return fail(ADJ_E_ARG, "autotune while live profiling is armed");
  hipStream_t st = (hipStream_t)stream;
  reps = std::max(1, reps);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ADJ_E_DEVICE, "hipEventCreate failed");
  }
  adj_status status = ADJ_OK;
  auto time_of = [&](const adj_tuning& t, float* out_ms) -> adj_status {
    s->tune = t;
    float bms = 1e30f;
    for (int r = 0; r < reps; ++r) {
      drop_chunk_graphs(s);
      if (hipEventRecord(e0, st) != hipSuccess) return fail(ADJ_E_DEVICE, "hipEventRecord failed");
      adj_solve_info info{};
      adj_status a = adjoint_solve(s, dL_dq, dL_dv, z, opts, &info, stream);
      if (a != ADJ_OK) return a;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return fail(ADJ_E_DEVICE, "event synchronisation failed");
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return fail(ADJ_E_DEVICE, "event timing failed");
      bms = std::min(bms, ms);
    }
    *out_ms = bms;
    return ADJ_OK;
  };
  adj_tuning cur = s->tune;
  float cur_ms = 0.f;
  status = time_of(cur, &cur_ms);
  const int gs[] = {64, 128, 256}, ln[] = {4, 8, 16, 32}, ch[] = {4, 8, 16, 32}, gr[] = {0, 1};
  for (int sweep = 0; sweep < 2 && status == ADJ_OK; ++sweep) {
    for (int dim = 0; dim < 4 && status == ADJ_OK; ++dim) {
      const int* vals = dim == 0 ? gs : dim == 1 ? ln : dim == 2 ? ch : gr;
      const int nvals = dim == 0 ? 3 : dim == 3 ? 2 : 4;
      for (int k = 0; k < nvals && status == ADJ_OK; ++k) {
        adj_tuning t = cur;
        int* field = dim == 0 ? &t.gs_rows : dim == 1 ? &t.bsr_lanes : dim == 2 ? &t.chunk : &t.graph;
        if (*field == vals[k]) continue;
        *field = vals[k];
        float ms = 0.f;
        status = time_of(t, &ms);
        if (status == ADJ_OK && ms < cur_ms) {
          cur = t;
          cur_ms = ms;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->tune = cur;
  drop_chunk_graphs(s);
  *best = cur;
  return status;
}

extern "C" adj_status adj_profile_begin(adj_scene* s, int32_t kernel) {
  if (!s || kernel < 0 || kernel > 12) return fail(ADJ_E_ARG, "bad profile request");
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
    case 6: src = s->cap_lu ? s->d_lu_P : nullptr; bytes = s->cap_lu ? (int64_t)s->mp * 128 * 8 : 0; break;
    default: return fail(ADJ_E_ARG, "unknown array");
  }
  *size_bytes = bytes;
  if (!host_out || capacity_bytes < bytes) return fail(ADJ_E_SHAPE, "buffer too small");
  HIPCHK(hipDeviceSynchronize());
  if (bytes) HIPCHK(hipMemcpy(host_out, src, bytes, hipMemcpyDeviceToHost));
  return ADJ_OK;
}

// ---------------------------------------------------------------------------
// Forward step (eq:dynamics).  Damped Newton on the step displacement u = q -
// qbar, the normal multipliers lambda_n and the friction magnitudes s
// (lambda_f = -s delta_f/|delta_f|).  The reduced Newton matrix is Acal at
// the iterate, assembled and solved with the adjoint's kernels (non-
// transposed).  Contact rows are O(n_c) and evaluated on the host; the
// per-tet and per-vertex work and the linear solves run on the GPU.
// ---------------------------------------------------------------------------

namespace {

inline double fb_rm(double x, double y, double e2) {  // r - x
  const double r = std::sqrt(x * x + y * y + e2);
  return (x > 0.0) ? (y * y + e2) / (r + x) : r - x;
}
inline double fb_phi(double x, double y, double e2) {
  const double r = std::sqrt(x * x + y * y + e2);
  const double sxy = x + y;
  return (sxy > 0.0) ? (2.0 * (x * y) - e2) / (sxy + r) : sxy - r;
}

struct FwdContacts {
  int n = 0;
  std::vector<int> vid, collider, fric;
  std::vector<double> frame, d_n, d_f, k, g0;
};

void tangent_frame(const double* n, double* F) {
  const double an[3] = {std::fabs(n[0]), std::fabs(n[1]), std::fabs(n[2])};
  int kk = 0;
  if (an[1] < an[kk]) kk = 1;
  if (an[2] < an[kk]) kk = 2;
  double e[3] = {0, 0, 0};
  e[kk] = 1.0;
  double c[3] = {n[1] * e[2] - n[2] * e[1], n[2] * e[0] - n[0] * e[2], n[0] * e[1] - n[1] * e[0]};
  const double nc = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  double t1[3] = {c[0] / nc, c[1] / nc, c[2] / nc};
  double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
  for (int i = 0; i < 3; ++i) {
    F[i] = n[i];
    F[3 + i] = t1[i];
    F[6 + i] = t2[i];
  }
}

// Contact state at (uc, lam_n, s): delta, |delta_f|, direction, lambda, phi rows.
struct CState {
  std::vector<double> delta, x, dhat, lam, phin, phif;
};

void contact_state(const FwdContacts& C, const std::vector<double>& uc, const std::vector<double>& lam_n,
                   const std::vector<double>& sf, double mu, const std::vector<double>& eps, CState& out) {
  const int n = C.n;
  out.delta.assign(3 * n, 0.0);
  out.x.assign(n, 0.0);
  out.dhat.assign(2 * n, 0.0);
  out.lam.assign(3 * n, 0.0);
  out.phin.assign(n, 0.0);
  out.phif.assign(n, 0.0);
  for (int c = 0; c < n; ++c) {
    const double* F = &C.frame[9 * c];
    const double* u = &uc[3 * c];
    const double dn = C.g0[c] + (F[0] * u[0] + F[1] * u[1] + F[2] * u[2]);
    const double d1 = (F[3] * u[0] + F[4] * u[1] + F[5] * u[2]) - C.d_f[2 * c];
    const double d2 = (F[6] * u[0] + F[7] * u[1] + F[8] * u[2]) - C.d_f[2 * c + 1];
    out.delta[3 * c] = dn;
    out.delta[3 * c + 1] = d1;
    out.delta[3 * c + 2] = d2;
    const double x = std::hypot(d1, d2);
    out.x[c] = x;
    double h1 = 1.0, h2 = 0.0;
    if (x > 0) {
      h1 = d1 / x;
      h2 = d2 / x;
    }
    out.dhat[2 * c] = h1;
    out.dhat[2 * c + 1] = h2;
    out.lam[3 * c] = lam_n[c];
    if (C.fric[c]) {
      out.lam[3 * c + 1] = -sf[c] * h1;
      out.lam[3 * c + 2] = -sf[c] * h2;
    }
    const double k = C.k[c];
    const double e2 = 2.0 * eps[c] * eps[c] * k;
    out.phin[c] = fb_phi(k * dn, lam_n[c], e2);
    out.phif[c] = C.fric[c] ? fb_phi(k * x, mu * lam_n[c] - sf[c], e2) : 0.0;
  }
}

}  // namespace

// Residual r_q (device, s->d_rq), contact state (host) and merit at (u_dev, lam_n, s).
static adj_status fwd_eval(adj_scene* s, hipStream_t st, const double* qbar, const double* u_dev,
                           const FwdContacts& C, const std::vector<double>& lam_n,
                           const std::vector<double>& sf, double mu, const std::vector<double>& eps,
                           CState& cs, double* merit, double* fmax, double* pmax, bool* inverted) {
  const double h = s->hs.h, h2 = h * h;
  const long long n3 = s->n3;
  launch_add_vec(st, n3, qbar, u_dev, 1.0, s->d_qcur);
  HIPCHK(hipMemsetAsync(s->d_err + 1, 0, sizeof(int), st));
  launch_tet_force(st, s->nt, s->d_tets, s->d_Bt, s->d_vol, s->d_lmu, s->d_llam, h2, s->d_qcur, s->d_force,
                   s->d_err, s->material);
  launch_gather_force(st, s->nv, s->d_vptr, s->d_vcode, s->d_force, s->d_mass, u_dev, s->d_utilde, s->d_rq);
  launch_binding_force(st, s->nb, s->d_bvid, s->d_bE, h2, s->d_qcur, s->d_btarget, s->d_rq);
  std::vector<double> uc(3 * (size_t)C.n);
  if (C.n) {
    launch_gather_contact_rows(st, C.n, s->d_fvid, u_dev, s->d_cu);
    HIPCHK(hipMemcpyAsync(uc.data(), s->d_cu, 3 * C.n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  contact_state(C, uc, lam_n, sf, mu, eps, cs);
  if (C.n) {
    std::vector<double> fw(3 * (size_t)C.n);
    for (int c = 0; c < C.n; ++c) {
      const double* F = &C.frame[9 * c];
      const double* l = &cs.lam[3 * c];
      for (int j = 0; j < 3; ++j) fw[3 * c + j] = -h2 * (F[j] * l[0] + F[3 + j] * l[1] + F[6 + j] * l[2]);
    }
    HIPCHK(hipMemcpyAsync(s->d_cvec, fw.data(), fw.size() * sizeof(double), hipMemcpyHostToDevice, st));
    launch_add_contact_vec(st, C.n, s->d_fvid, s->d_cvec, s->d_rq);
  }
  launch_norms(st, n3, s->d_rq, s->P3(), s->d_norms);
  double nr[2];
  int errs[2];
  HIPCHK(hipMemcpyAsync(nr, s->d_norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(errs, s->d_err, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *inverted = errs[1] != 0;
  double ps = 0.0, pm = 0.0;
  for (int c = 0; c < C.n; ++c) {
    ps += cs.phin[c] * cs.phin[c] + cs.phif[c] * cs.phif[c];
    pm = std::max(pm, std::max(std::fabs(cs.phin[c]), std::fabs(cs.phif[c])));
  }
  *merit = 0.5 * (nr[0] / (h2 * h2) + ps);
  *fmax = nr[1] / h2;
  *pmax = pm;
  return ADJ_OK;
}

// One damped Newton solve with smoothing eps (per contact).  Returns ok.
static adj_status fwd_newton(adj_scene* s, hipStream_t st, const double* qbar, FwdContacts& C,
                             std::vector<double>& lam_n, std::vector<double>& sf, double mu,
                             const std::vector<double>& eps, int maxit, double tol_f, double tol_p,
                             bool* ok_out, int* iters) {
  const double h = s->hs.h, h2 = h * h;
  const long long n3 = s->n3;
  const int nc = C.n;
  CState cs;
  double merit, fmax, pmax;
  bool inv;
  adj_status a = fwd_eval(s, st, qbar, s->d_fu, C, lam_n, sf, mu, eps, cs, &merit, &fmax, &pmax, &inv);
  if (a != ADJ_OK) return a;
  if (inv) return fail(ADJ_E_INVERTED, "inverted element at the initial guess of the step");
  bool ok = false;
  int it = 0;
  std::vector<double> Wt(9 * (size_t)nc), Q(9 * (size_t)nc), kh(4 * (size_t)nc), rc(3 * (size_t)nc),
      av(nc), bv(nc), bn(nc), bf(nc);
  for (it = 1; it <= maxit; ++it) {
    // Newton matrix: elastic blocks at q = qbar + u, contact blocks at the iterate
    launch_add_vec(st, n3, qbar, s->d_fu, 1.0, s->d_qcur);
    launch_tet_blocks(st, s->nt, s->d_tets, s->d_Bt, s->d_vol, s->d_lmu, s->d_llam, h2, s->d_qcur,
                      s->d_tetblk, s->d_err, s->material);
    launch_assemble(st, s->nnzb, s->nt, s->d_slot_ptr, s->d_slot_code, s->d_tetblk, s->d_row_of_slot, s->d_col,
                    s->d_mass, s->d_val);
    launch_binding_fold(st, s->nb, s->d_bvid, s->d_bE, h2, s->d_diag_slot, s->d_val);
    for (int c = 0; c < nc; ++c) {
      const double k = C.k[c];
      const double e2 = 2.0 * eps[c] * eps[c] * k;
      const double dn = cs.delta[3 * c], x = cs.x[c];
      const double ra = fb_rm(k * dn, lam_n[c], e2), rb = fb_rm(lam_n[c], k * dn, e2);
      const double rn = std::sqrt((k * dn) * (k * dn) + lam_n[c] * lam_n[c] + e2);
      av[c] = k * ra / rb;
      bn[c] = rb / rn;
      double Rm[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
      double Kh[3][3] = {{av[c], 0, 0}, {0, 0, 0}, {0, 0, 0}};
      bv[c] = 0.0;
      bf[c] = 1.0;
      double cc = 0.0;
      if (C.fric[c]) {
        const double yf = mu * lam_n[c] - sf[c];
        const double rfa = fb_rm(k * x, yf, e2), rfb = fb_rm(yf, k * x, e2);
        const double rf = std::sqrt((k * x) * (k * x) + yf * yf + e2);
        bv[c] = k * rfa / rfb;
        bf[c] = rfb / rf;
        cc = (x > 0) ? sf[c] / x : 0.0;
        const double h1 = cs.dhat[2 * c], hh2 = cs.dhat[2 * c + 1];
        Rm[1][1] = h1; Rm[1][2] = hh2; Rm[2][1] = -hh2; Rm[2][2] = h1;
        Kh[1][0] = -mu * av[c];
        Kh[1][1] = bv[c];
        Kh[2][2] = cc;
      }
      // K = R^T Kh R (frame coordinates); world block h^2 F^T K F; Q = R F
      double T[3][3], K[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[i][j] = Kh[i][0] * Rm[0][j] + Kh[i][1] * Rm[1][j] + Kh[i][2] * Rm[2][j];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K[i][j] = Rm[0][i] * T[0][j] + Rm[1][i] * T[1][j] + Rm[2][i] * T[2][j];
      const double* F = &C.frame[9 * c];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double acc = 0.0;
          for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) acc += F[3 * p + i] * K[p][q] * F[3 * q + j];
          Wt[9 * c + 3 * i + j] = h2 * acc;
          Q[9 * c + 3 * i + j] = Rm[i][0] * F[j] + Rm[i][1] * F[3 + j] + Rm[i][2] * F[6 + j];
        }
      kh[4 * c] = av[c];
      kh[4 * c + 1] = bv[c];
      kh[4 * c + 2] = cc;
      kh[4 * c + 3] = C.fric[c] ? 1.0 : 0.0;
      // rhs contribution h^2 F^T R^T e
      double e[3] = {-cs.phin[c] / bn[c], 0.0, 0.0};
      if (C.fric[c]) e[1] = mu * cs.phin[c] / bn[c] - cs.phif[c] / bf[c];
      double re[3];
      for (int i = 0; i < 3; ++i) re[i] = Rm[0][i] * e[0] + Rm[1][i] * e[1] + Rm[2][i] * e[2];
      for (int j = 0; j < 3; ++j) rc[3 * c + j] = h2 * (F[j] * re[0] + F[3 + j] * re[1] + F[6 + j] * re[2]);
    }
    if (nc) {
      HIPCHK(hipMemcpyAsync(s->d_Wt, Wt.data(), Wt.size() * sizeof(double), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(s->d_Q, Q.data(), Q.size() * sizeof(double), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(s->d_kh, kh.data(), kh.size() * sizeof(double), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(s->d_cvec, rc.data(), rc.size() * sizeof(double), hipMemcpyHostToDevice, st));
      launch_contact_fold(st, nc, s->d_fvid, s->d_diag_slot, s->d_Wt, s->d_val);
      if ((a = build_capacitance(s, st, mu, 0)) != ADJ_OK) return a;
    }
    launch_bsr_soa(st, s->nnzb, s->d_val, s->d_valT, nullptr);  // the Krylov products' copy
    // rhs = -r_q + h^2 sum F^T R^T e
    launch_scale_vec(st, n3, s->d_rq, -1.0, s->d_rhs);
    launch_add_contact_vec(st, nc, s->d_fvid, s->d_cvec, s->d_rhs);
    int git = 0;
    double grel = 0.0;
    bool gconv = false;
    if ((a = gmres_solve(s, st, s->d_rhs, s->d_du, 1e-11, 600, 64, &git, &grel, &gconv)) != ADJ_OK) return a;
    // multiplier updates
    std::vector<double> duc(3 * (size_t)nc), dlam(nc), ds(nc), ddf(2 * (size_t)nc);
    if (nc) {
      launch_gather_contact_rows(st, nc, s->d_fvid, s->d_du, s->d_cu);
      HIPCHK(hipMemcpyAsync(duc.data(), s->d_cu, duc.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    for (int c = 0; c < nc; ++c) {
      const double* F = &C.frame[9 * c];
      const double* d = &duc[3 * c];
      const double ddn = F[0] * d[0] + F[1] * d[1] + F[2] * d[2];
      ddf[2 * c] = F[3] * d[0] + F[4] * d[1] + F[5] * d[2];
      ddf[2 * c + 1] = F[6] * d[0] + F[7] * d[1] + F[8] * d[2];
      dlam[c] = -av[c] * ddn - cs.phin[c] / bn[c];
      if (C.fric[c]) {
        const double dx = cs.dhat[2 * c] * ddf[2 * c] + cs.dhat[2 * c + 1] * ddf[2 * c + 1];
        ds[c] = mu * dlam[c] + bv[c] * dx + cs.phif[c] / bf[c];
      } else {
        ds[c] = 0.0;
      }
    }
    // no step may shrink |delta_f| of a frictional contact below 1% of its value
    double alpha = 1.0;
    for (int k = 0; k < 60; ++k) {
      bool viol = false;
      for (int c = 0; c < nc && !viol; ++c) {
        if (!C.fric[c] || !(cs.x[c] > 0)) continue;
        const double x1 = cs.delta[3 * c + 1] + alpha * ddf[2 * c];
        const double x2 = cs.delta[3 * c + 2] + alpha * ddf[2 * c + 1];
        if (std::hypot(x1, x2) < 0.01 * cs.x[c]) viol = true;
      }
      if (!viol) break;
      alpha *= 0.5;
    }
    bool accepted = false;
    CState ct;
    double mt = 0, ft = 0, pt = 0;
    std::vector<double> lt(nc), stt(nc);
    for (int k = 0; k < 40; ++k) {
      launch_add_vec(st, n3, s->d_fu, s->d_du, alpha, s->d_ut);
      for (int c = 0; c < nc; ++c) {
        lt[c] = lam_n[c] + alpha * dlam[c];
        stt[c] = sf[c] + alpha * ds[c];
      }
      if ((a = fwd_eval(s, st, qbar, s->d_ut, C, lt, stt, mu, eps, ct, &mt, &ft, &pt, &inv)) != ADJ_OK) return a;
      if (inv) {
        alpha *= 0.5;
        continue;
      }
      if (mt <= (1.0 - 1e-4 * alpha) * merit || mt == 0.0) {
        accepted = true;
        break;
      }
      alpha *= 0.5;
    }
    if (!accepted) break;
    // accept: u <- u_trial
    HIPCHK(hipMemcpyAsync(s->d_fu, s->d_ut, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
    lam_n = lt;
    sf = stt;
    cs = ct;
    const double prev = merit;
    merit = mt;
    fmax = ft;
    pmax = pt;
    // |alpha du|_max and |u|_max for the small-step test
    launch_scale_vec(st, n3, s->d_du, alpha, s->d_ut);
    launch_norms(st, n3, s->d_ut, s->P3(), s->d_norms);
    double nd[2], nu[2];
    HIPCHK(hipMemcpyAsync(nd, s->d_norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    launch_norms(st, n3, s->d_fu, s->P3(), s->d_norms);
    HIPCHK(hipMemcpyAsync(nu, s->d_norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const bool small = nd[1] <= 4e-16 * std::max(1.0, nu[1]);
    if (alpha == 1.0 && ((fmax <= tol_f && pmax <= tol_p) || small)) {
      ok = fmax <= 1e3 * tol_f && pmax <= 1e3 * tol_p;
      break;
    }
    // rounding floor: within 1e3 of the tolerances and the step no longer
    // halves the residual (the merit is its square)
    if (fmax <= 1e3 * tol_f && pmax <= 1e3 * tol_p && merit > 0.25 * prev) {
      ok = true;
      break;
    }
  }
  if (!ok) ok = fmax <= 1e3 * tol_f && pmax <= 1e3 * tol_p;
  *ok_out = ok;
  *iters = it;
  return ADJ_OK;
}

extern "C" adj_status sim_forward_step(adj_scene* s, const double* qbar, const double* vbar,
                                       const double* f_ext, double mu, double* q, double* v,
                                       adj_contact_state* out, void* stream) {
  if (!s || !qbar || !vbar || !f_ext || !q || !v || !out) return fail(ADJ_E_ARG, "null argument");
  if (!std::isfinite(mu) || mu < 0) return fail(ADJ_E_ARG, "mu must be finite and >= 0");
  if (s->nb && !s->btarget_set) return fail(ADJ_E_ARG, "binding targets not set (adj_set_binding_targets)");
  hipStream_t st = (hipStream_t)stream;
  const double h = s->hs.h;
  const long long n3 = s->n3;
  const int np = (int)(s->hs.planes.size() / 4);
  const int ns = s->n_spheres;
  if (np + ns > 15) return fail(ADJ_E_ARG, "at most 15 colliders (planes and spheres)");
  // prediction and candidates
  launch_fwd_predict(st, s->nv, qbar, vbar, f_ext, s->d_mass, h, s->hs.gravity, s->d_utilde, s->d_qtilde);
  launch_fwd_detect(st, s->nv, qbar, s->d_qtilde, np, s->d_planes, ns, s->d_sph, s->d_sph + 4 * ns, s->hs.margin,
                    s->d_mask);
  std::vector<int> mask(s->nv);
  HIPCHK(hipMemcpyAsync(mask.data(), s->d_mask, s->nv * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  FwdContacts C;
  std::vector<int> sph_rows;  // contacts with a sphere: their frames follow below
  for (int vv = 0; vv < s->nv; ++vv)
    for (int p = 0; p < np + ns; ++p)
      if (mask[vv] & (1 << (2 * p))) {
        C.vid.push_back(vv);
        C.collider.push_back(p);
        C.fric.push_back((mask[vv] >> (2 * p + 1)) & 1);
        double F[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (p < np) {
          tangent_frame(&s->hs.planes[4 * p], F);
          C.d_n.push_back(s->hs.planes[4 * p + 3]);
        } else {
          sph_rows.push_back((int)C.vid.size() - 1);
          C.d_n.push_back(0.0);
        }
        C.frame.insert(C.frame.end(), F, F + 9);
        C.d_f.push_back(0.0);
        C.d_f.push_back(0.0);
        C.k.push_back(s->hs.As[s->hs.diag_slot[vv]] / (h * h));
      }
  C.n = (int)C.vid.size();
  const int nc = C.n;
  if (nc > s->max_contacts || nc > out->capacity)
    return fail(ADJ_E_SHAPE, "more contacts than max_contacts / the output capacity");
  if (!sph_rows.empty()) {
    // frames of the sphere contacts from qbar (the same expressions as the
    // detection kernel, evaluated left to right)
    std::vector<int> rows_v(sph_rows.size());
    for (size_t i = 0; i < sph_rows.size(); ++i) rows_v[i] = C.vid[sph_rows[i]];
    HIPCHK(hipMemcpyAsync(s->d_fvid, rows_v.data(), rows_v.size() * sizeof(int), hipMemcpyHostToDevice, st));
    launch_gather_contact_rows(st, (int)rows_v.size(), s->d_fvid, qbar, s->d_cu);
    std::vector<double> xs(3 * rows_v.size());
    HIPCHK(hipMemcpyAsync(xs.data(), s->d_cu, xs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (size_t i = 0; i < sph_rows.size(); ++i) {
      const int c = sph_rows[i], sp = C.collider[c] - np;
      const double* c0 = &s->sph[4 * sp];
      const double* c1 = &s->sph[4 * (ns + sp)];
      const double d0 = xs[3 * i] - c0[0], d1 = xs[3 * i + 1] - c0[1], d2 = xs[3 * i + 2] - c0[2];
      const double nrm = std::sqrt((d0 * d0 + d1 * d1) + d2 * d2);
      const double n[3] = {d0 / nrm, d1 / nrm, d2 / nrm};
      double* F = &C.frame[9 * (size_t)c];
      tangent_frame(n, F);
      C.d_n[c] = ((n[0] * c1[0] + n[1] * c1[1]) + n[2] * c1[2]) + c1[3];
      const double dc[3] = {c1[0] - c0[0], c1[1] - c0[1], c1[2] - c0[2]};
      C.d_f[2 * c] = (F[3] * dc[0] + F[4] * dc[1]) + F[5] * dc[2];
      C.d_f[2 * c + 1] = (F[6] * dc[0] + F[7] * dc[1]) + F[8] * dc[2];
    }
  }
  if (nc && (!out->vid || !out->fric || !out->frame || !out->delta || !out->lambda))
    return fail(ADJ_E_ARG, "contact output arrays missing");
  // gap at the start of the step, n . xbar - d_n
  C.g0.assign(nc, 0.0);
  if (nc) {
    HIPCHK(hipMemcpyAsync(s->d_fvid, C.vid.data(), nc * sizeof(int), hipMemcpyHostToDevice, st));
    launch_gather_contact_rows(st, nc, s->d_fvid, qbar, s->d_cu);
    std::vector<double> xb(3 * (size_t)nc);
    HIPCHK(hipMemcpyAsync(xb.data(), s->d_cu, xb.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int c = 0; c < nc; ++c)
      C.g0[c] = (C.frame[9 * c] * xb[3 * c] + C.frame[9 * c + 1] * xb[3 * c + 1] +
                 C.frame[9 * c + 2] * xb[3 * c + 2]) - C.d_n[c];
  }
  // warm start from the previous step (by vertex and collider)
  std::vector<double> lam0(nc, 0.0), s0(nc, 0.0);
  for (int c = 0; c < nc; ++c) {
    auto it = s->warm.find((long long)C.vid[c] * 64 + C.collider[c]);
    if (it != s->warm.end()) {
      lam0[c] = it->second.first;
      s0[c] = C.fric[c] ? it->second.second : 0.0;
    }
  }
  adj_status a = contact_layout(s, st, nc, C.vid, C.fric, true);
  if (a != ADJ_OK) return a;
  s->cur_vid = s->d_fvid;
  const double tol_f = 1e-11, tol_p = 1e-13;
  std::vector<double> lam_n = lam0, sf = s0;
  HIPCHK(hipMemcpyAsync(s->d_fu, s->d_utilde, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  int total = 0;
  while (true) {
    std::vector<double> l_start = lam_n, s_start = sf;
    // qtilde is free after detection: it keeps the starting displacement
    HIPCHK(hipMemcpyAsync(s->d_qtilde, s->d_fu, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
    std::vector<double> eps(nc, s->hs.eps);
    bool ok = false;
    int its = 0;
    if ((a = fwd_newton(s, st, qbar, C, lam_n, sf, mu, eps, 60, tol_f, tol_p, &ok, &its)) != ADJ_OK) return a;
    total += its;
    if (!ok) {
      // continuation in the smoothing: eps_j^2 = eps^2 gamma_j, gamma_j -> 1
      lam_n = l_start;
      sf = s_start;
      HIPCHK(hipMemcpyAsync(s->d_fu, s->d_qtilde, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
      for (double gamma = 1e6;; gamma /= 30.0) {
        const bool last = gamma <= 1.0;
        std::vector<double> ej(nc, s->hs.eps * std::sqrt(std::max(gamma, 1.0)));
        if ((a = fwd_newton(s, st, qbar, C, lam_n, sf, mu, ej, 60, last ? tol_f : 1e-7, last ? tol_p : 1e-7,
                            &ok, &its)) != ADJ_OK)
          return a;
        total += its;
        if (last) break;
      }
    }
    bool bad = false;
    for (int c = 0; c < nc; ++c)
      if (C.fric[c] && sf[c] < 0.0) {
        C.fric[c] = 0;
        sf[c] = 0.0;
        bad = true;
      }
    if (!bad) break;
    // a contact that separated inside the step has no solution of the
    // friction rows: demote it to normal-only and solve again
    if ((a = contact_layout(s, st, nc, C.vid, C.fric, true)) != ADJ_OK) return a;
  }
  // final state, record, outputs
  CState cs;
  double merit, fmax, pmax;
  bool inv;
  std::vector<double> eps(nc, s->hs.eps);
  if ((a = fwd_eval(s, st, qbar, s->d_fu, C, lam_n, sf, mu, eps, cs, &merit, &fmax, &pmax, &inv)) != ADJ_OK)
    return a;
  launch_add_vec(st, n3, qbar, s->d_fu, 1.0, q);
  launch_scale_vec(st, n3, s->d_fu, 1.0 / h, v);
  out->n_contacts = nc;
  out->mu = mu;
  if (nc) {
    HIPCHK(hipMemcpyAsync(out->vid, C.vid.data(), nc * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(out->fric, C.fric.data(), nc * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(out->frame, C.frame.data(), 9 * nc * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(out->delta, cs.delta.data(), 3 * nc * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(out->lambda, cs.lam.data(), 3 * nc * sizeof(double), hipMemcpyHostToDevice, st));
    if (out->d_n) HIPCHK(hipMemcpyAsync(out->d_n, C.d_n.data(), nc * sizeof(double), hipMemcpyHostToDevice, st));
    if (out->d_f) HIPCHK(hipMemcpyAsync(out->d_f, C.d_f.data(), 2 * nc * sizeof(double), hipMemcpyHostToDevice, st));
  }
  s->warm.clear();
  for (int c = 0; c < nc; ++c) s->warm[(long long)C.vid[c] * 64 + C.collider[c]] = {lam_n[c], sf[c]};
  HIPCHK(hipStreamSynchronize(st));
  s->fwd_newton_iters = total;
  s->fwd_residual = std::max(fmax, pmax);
  s->setup_done = false;  // the adjoint workspaces now hold the Newton matrix
  // the paper's (unscaled) rows at the returned state
  double worst = fmax;
  for (int c = 0; c < nc; ++c) {
    const double e2 = 2.0 * s->hs.eps * s->hs.eps;
    worst = std::max(worst, std::fabs(fb_phi(cs.delta[3 * c], cs.lam[3 * c], e2)));
    if (C.fric[c]) worst = std::max(worst, std::fabs(fb_phi(cs.x[c], mu * lam_n[c] - sf[c], e2)));
  }
  s->fwd_residual = worst;
  if (!(worst <= 1e-8)) return fail(ADJ_E_NOCONV, "forward Newton residual " + std::to_string(worst));
  return ADJ_OK;
}

extern "C" adj_status adj_set_actuation(adj_scene* s, int32_t n_groups, const int32_t* group, const double* fibre) {
  if (!s) return fail(ADJ_E_ARG, "scene is null");
  if (n_groups < 1 || n_groups > 65536 || !group || !fibre) return fail(ADJ_E_ARG, "invalid actuation groups");
  std::vector<int> gptr(n_groups + 1, 0), gtets(s->nt);
  for (int t = 0; t < s->nt; ++t) {
    if (group[t] < 0 || group[t] >= n_groups) return fail(ADJ_E_ARG, "actuation group out of range");
    const double* d = fibre + 3 * (size_t)t;
    if (!std::isfinite(d[0]) || !std::isfinite(d[1]) || !std::isfinite(d[2])) return fail(ADJ_E_ARG, "non-finite fibre");
    gptr[group[t] + 1]++;
  }
  for (int g = 0; g < n_groups; ++g) gptr[g + 1] += gptr[g];
  {
    std::vector<int> fill(gptr.begin(), gptr.end() - 1);
    for (int t = 0; t < s->nt; ++t) gtets[fill[group[t]]++] = t;  // tets of a group in index order
  }
  HIPCHK(hipDeviceSynchronize());  // earlier actuation calls may still read the old tables
  for (void* p : {(void*)s->d_act_group, (void*)s->d_act_gptr, (void*)s->d_act_gtets, (void*)s->d_act_fibre,
                  (void*)s->d_act12, (void*)s->d_act_s})
    if (p) HIPCHK(hipFree(p));
  s->d_act_group = s->d_act_gptr = s->d_act_gtets = nullptr;
  s->d_act_fibre = s->d_act12 = s->d_act_s = nullptr;
  s->n_act = 0;
  const size_t nt = (size_t)s->nt;
  if (hipMalloc(&s->d_act_group, nt * sizeof(int)) != hipSuccess ||
      hipMalloc(&s->d_act_gptr, (n_groups + 1) * sizeof(int)) != hipSuccess ||
      hipMalloc(&s->d_act_gtets, nt * sizeof(int)) != hipSuccess ||
      hipMalloc(&s->d_act_fibre, 3 * nt * sizeof(double)) != hipSuccess ||
      hipMalloc(&s->d_act12, 12 * nt * sizeof(double)) != hipSuccess ||
      hipMalloc(&s->d_act_s, nt * sizeof(double)) != hipSuccess)
    return fail(ADJ_E_OOM, "actuation tables");
  HIPCHK(hipMemcpy(s->d_act_group, group, nt * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->d_act_gptr, gptr.data(), (n_groups + 1) * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->d_act_gtets, gtets.data(), nt * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->d_act_fibre, fibre, 3 * nt * sizeof(double), hipMemcpyHostToDevice));
  s->n_act = n_groups;
  return ADJ_OK;
}

extern "C" adj_status adj_actuation_force(adj_scene* s, const double* a, double* f, void* stream) {
  if (!s || !a || !f) return fail(ADJ_E_ARG, "null argument");
  if (!s->n_act) return fail(ADJ_E_ARG, "adj_set_actuation has not run on this scene");
  launch_actuation_force((hipStream_t)stream, s->nt, s->nv, s->d_act_group, s->d_act_fibre, s->d_Bt, s->d_vol,
                         s->d_vptr, s->d_vcode, a, s->d_act12, f);
  HIPCHK(hipGetLastError());
  return ADJ_OK;
}

extern "C" adj_status adj_actuation_vjp(adj_scene* s, const double* dL_df, double* dL_da, void* stream) {
  if (!s || !dL_df || !dL_da) return fail(ADJ_E_ARG, "null argument");
  if (!s->n_act) return fail(ADJ_E_ARG, "adj_set_actuation has not run on this scene");
  launch_actuation_vjp((hipStream_t)stream, s->nt, s->n_act, s->d_tets, s->d_act_fibre, s->d_Bt, s->d_vol,
                       s->d_act_gptr, s->d_act_gtets, dL_df, s->d_act_s, dL_da);
  HIPCHK(hipGetLastError());
  return ADJ_OK;
}

extern "C" adj_status adj_set_binding_targets(adj_scene* s, const double* targets) {
  if (!s) return fail(ADJ_E_ARG, "scene is null");
  if (!s->nb) return fail(ADJ_E_ARG, "the scene has no bindings");
  if (!targets) return fail(ADJ_E_ARG, "null targets");
  for (int i = 0; i < 3 * s->nb; ++i)
    if (!std::isfinite(targets[i])) return fail(ADJ_E_ARG, "non-finite binding target");
  HIPCHK(hipMemcpy(s->d_btarget, targets, 3 * (size_t)s->nb * sizeof(double), hipMemcpyHostToDevice));
  s->btarget_set = true;
  return ADJ_OK;
}

extern "C" adj_status adj_set_spheres(adj_scene* s, int32_t n, const double* old_pose, const double* new_pose) {
  if (!s) return fail(ADJ_E_ARG, "scene is null");
  if (n < 0 || (n > 0 && (!old_pose || !new_pose))) return fail(ADJ_E_ARG, "sphere poses missing");
  const int np = (int)(s->hs.planes.size() / 4);
  if (np + n > 15) return fail(ADJ_E_ARG, "at most 15 colliders (planes and spheres)");
  for (int i = 0; i < 4 * n; ++i)
    if (!std::isfinite(old_pose[i]) || !std::isfinite(new_pose[i])) return fail(ADJ_E_ARG, "non-finite pose");
  for (int i = 0; i < n; ++i)
    if (!(new_pose[4 * i + 3] > 0)) return fail(ADJ_E_ARG, "sphere radius must be positive");
  if (n > s->sph_cap) {
    if (s->d_sph) HIPCHK(hipFree(s->d_sph));
    s->d_sph = nullptr;
    s->sph_cap = 0;
    if (hipMalloc(&s->d_sph, 8 * (size_t)n * sizeof(double)) != hipSuccess) return fail(ADJ_E_OOM, "spheres");
    s->sph_cap = n;
  }
  s->sph.assign(old_pose, old_pose + 4 * n);
  s->sph.insert(s->sph.end(), new_pose, new_pose + 4 * n);
  if (n > 0) HIPCHK(hipMemcpy(s->d_sph, s->sph.data(), 8 * (size_t)n * sizeof(double), hipMemcpyHostToDevice));
  s->n_spheres = n;
  return ADJ_OK;
}

extern "C" adj_status adj_forward_stats(const adj_scene* s, double* out) {
  if (!s || !out) return fail(ADJ_E_ARG, "null argument");
  out[0] = s->fwd_newton_iters;
  out[1] = s->fwd_residual;
  return ADJ_OK;
}

extern "C" adj_status adj_forward_reset(adj_scene* s) {
  if (!s) return fail(ADJ_E_ARG, "scene is null");
  s->warm.clear();
  return ADJ_OK;
}

#include "api_batch.inc"
