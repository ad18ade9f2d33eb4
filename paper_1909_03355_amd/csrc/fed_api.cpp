// C ABI of the FED-FEM library (see include/fedfem.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/fedfem.h"
#include "fed_internal.h"
#include "fed_kernels.h"

namespace {

thread_local std::string g_err;

// static LDS of the step kernels' energy check (block sums and a flag),
// reserved out of the LDS a tile may take
constexpr int kStaticLds = 512;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(FED_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),  \
                  __FILE__, __LINE__);                                                \
  } while (0)

// device allocations of a context, freed together: from the caller's
// allocator hooks when given (fed_options.dev_alloc / dev_free), else
// hipMalloc / hipFree
struct DevPool {
  void *(*af)(size_t, void *) = nullptr;
  void (*ff)(void *, void *) = nullptr;
  void *actx = nullptr;
  std::vector<void *> ptrs;
  std::vector<size_t> sizes;
  size_t total = 0;  // bytes held
  hipError_t alloc(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    if (af) {
      *p = af(bytes, actx);
      if (!*p) return hipErrorOutOfMemory;
    } else {
      hipError_t e = hipMalloc(p, bytes);
      if (e != hipSuccess) return e;
    }
    ptrs.push_back(*p);
    sizes.push_back(bytes);
    total += bytes;
    return hipSuccess;
  }
  void give_back(void *p) {
    if (ff) ff(p, actx);
    else (void)hipFree(p);
  }
  // gives one buffer back; with the caller's hooks the device is synchronised
  // first (hipFree does that itself), so no enqueued work still uses it
  void release(void *p) {
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
      if (af) (void)hipDeviceSynchronize();
      give_back(p);
      const size_t i = (size_t)(it - ptrs.begin());
      total -= sizes[i];
      sizes.erase(sizes.begin() + i);
      ptrs.erase(it);
    }
  }
  void free_all() {
    for (void *p : ptrs) give_back(p);
    ptrs.clear();
    sizes.clear();
    total = 0;
  }
};

}  // namespace

namespace fed {
// work arrays of the adjoint: the states of the segment at hand (ckpt_every + 1
// hi vectors and two lo), the multiplier pair (hi, lo) ping-pong, the FP64
// boundary and derivative sums, 1/dt per node and rho V / n_e per element
struct AdjWork {
  void *seg = nullptr, *lamb[2] = {nullptr, nullptr}, *rdt = nullptr, *mV = nullptr;
  float *seglo[2] = {nullptr, nullptr}, *lamlo[2] = {nullptr, nullptr};
  double *S0 = nullptr, *S1 = nullptr, *gk = nullptr, *gc = nullptr, *gh = nullptr;
};
}  // namespace fed

struct fed_ctx {
  int prec = 0, ne = 8, rb = 4;
  int64_t N = 0, E = 0, Eexp = 0, nrec = 0, ninst = 1, ndir = 0;
  fed::Tiling til;
  DevPool pool;
  // step working set
  fed::TileHdr *d_tiles = nullptr;
  uint16_t *d_ent = nullptr;
  int32_t *d_halo = nullptr, *d_perm = nullptr, *d_eorig = nullptr, *d_rec_of = nullptr;
  uint8_t *d_eowner = nullptr;
  void *d_H = nullptr, *d_alpha = nullptr, *d_beta = nullptr;
  void *d_rA = nullptr, *d_rAT = nullptr, *d_reA = nullptr, *d_rTa = nullptr, *d_rP = nullptr;
  void *d_T[2] = {nullptr, nullptr};
  float *d_lo[2] = {nullptr, nullptr};
  int32_t *d_dir_node = nullptr;
  double *d_dir_T = nullptr;
  int *d_flag = nullptr;
  double *d_Tuser = nullptr;  // FP64 staging in caller order
  // resident stepping: exported nodes, tagged exchange buffers, the next tag,
  // the wait-error flag
  bool resident = false;
  uint8_t *d_exported = nullptr;
  unsigned long long *d_X[2] = {nullptr, nullptr};
  unsigned xtag = 1;
  int *d_rerr = nullptr;
  int res_lds = 0;
  bool res_nv = false;     // resident table laws: the table's values at the nodes in LDS
  bool res_oph = false;    // resident uniform-gradient hexahedron: halo elements' operators in LDS
  int64_t res_oph_elems = 0;  // (expanded) elements whose operators stay in LDS
  int16_t *d_sigma = nullptr;  // resident LDS positions of the touched nodes (or null)
  uint16_t *d_ent_sigma = nullptr;  // the packed entries with those positions
  int res_sstride = 0;
  // bounded halo waits of resident launches; tag_skew != 0 only in tests of
  // the failure path (fed_test_waits)
  int spin_limit = 1 << 22;
  unsigned tag_skew = 0;
  int res_split = 1;  // resident steps run the tile-interior elements during the halo wait
  // resident adjoint (hexahedra, folded operator, tiles within the LDS)
  bool adjres = false;
  int adjres_lds = 0;
  // kept FP64 pre-computation (re-derived by fed_set_params, used by the adjoint)
  double *d_H0 = nullptr, *d_kscale = nullptr, *d_V = nullptr;
  double *d_M0 = nullptr, *d_M1 = nullptr, *d_Cmin = nullptr, *d_lamgeo = nullptr;
  double *d_ec0 = nullptr;  // per-element heat capacity override (fed_set_params)
  fed::MatDev *d_mats = nullptr;
  int32_t *d_emat = nullptr, *d_ince = nullptr, *d_einst = nullptr, *d_ninst = nullptr;
  int64_t *d_incp = nullptr;
  int32_t *d_faces = nullptr, *d_recitem = nullptr, *d_recnode = nullptr;
  int64_t *d_recptr = nullptr;
  double *d_fh = nullptr, *d_fTa = nullptr, *d_feps = nullptr, *d_fq = nullptr, *d_farea = nullptr;
  double *d_ptW = nullptr, *d_b64[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  // point-load schedule: its rows of concentrated loads (FP64, npt each) and
  // the record powers of every row (step precision, nrec each)
  double *d_psW = nullptr;
  void *d_psP = nullptr;
  int64_t ps_rows = 0;
  double *d_dtinst = nullptr;
  uint8_t *d_isdir = nullptr;
  unsigned long long *d_lam = nullptr;
  int64_t nf = 0, npt = 0;
  int nfn = 4;
  // host copy of the faces and their emissivities (radiation ambients must
  // stay single-valued per node when fed_set_bc changes them)
  std::vector<int32_t> h_faces;
  std::vector<double> h_feps;
  bool has_rad = false, allow_unstable = false;
  // checkpoints (state after every ckpt_every steps) and adjoint work arrays
  int64_t ckpt_every = 0;
  std::vector<void *> ck_hi, ck_lo;
  // kept states (resident contexts, fed_keep_states): per checkpoint segment
  // g the hi of steps g*ckpt_every .. (g+1)*ckpt_every, written by the forward
  // launches, so fed_backward need not recompute them; kept_ok while every
  // step since fed_set_temperature was stored
  bool keep_states = false, kept_ok = false;
  std::vector<void *> segbuf;
  fed::AdjWork adjw;  // fed_backward's work arrays (allocated on first use)
  int adj_lds = 0, max_lds = 64 * 1024;
  // conductivity/capacity laws: per-element (s0, s1) when the materials differ,
  // shared multiplier tables (step precision) and their extremes on [T_lo, T_hi]
  void *d_esk = nullptr, *d_ktab = nullptr, *d_ctab = nullptr;
  int nkt = 0, nct = 0;
  double fk_max = 1.0, fc_min = 1.0;
  // element operator: 0 the folded 3x3 (6 values), 1 the uniform-gradient
  // hexahedron (27 values)
  int op = 0, hw = 6;
  double hg_eps = 0;  // hourglass control of the uniform-gradient hexahedron (op 2)
  // rows of H that take the per-element conductivity factor: V D, and kappa
  int hs_from() const { return op ? 21 : 0; }
  int hs_to() const { return op == 2 ? 28 : hw; }
  // host copies for re-deriving the stability bound over a new range
  std::vector<fed_material> h_mats;
  std::vector<double> h_ktab_T, h_ktab_f, h_ctab_T, h_ctab_f;
  // in-run health check: the record the step kernels write, per-tile partial
  // sums of the energy checks, the window margin, the energy-check interval
  // (0: the last step of every fed_step call) and the energy tolerance (0: report only)
  fed::Health *d_health = nullptr;
  double *d_hpart = nullptr;
  double check_margin = 0, energy_tol = 0;
  int check_window = 0;             // 0: derived from the stability bound, 1: the margin
  double win_lo = 0, win_hi = 0;    // the window in use
  int64_t check_every = 0;
  unsigned long long *d_rkeys = nullptr;  // temperature-range keys and a non-finite flag
  int *d_rnan = nullptr;
  // scalars
  double s0 = 1, s1 = 0, Tz = -273.15, T_lo = 0, T_hi = 0;
  int tdk = 0, tdc = 0, block = 256, nper = 1, K = 1;
  std::vector<double> dt_crit, dt_used;
  int cur = 0;
  int64_t steps = 0;
  bool have_T = false;
  // graph of captured steps
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream the graph is captured on
  int gsteps = 0, gparity = -1;
  fed_info info{};

  fed::StepArgs step_args(int parity, int k) const {
    fed::StepArgs a{};
    a.prec = prec;
    a.ne = ne;
    a.k = k;
    a.tdk = tdk;
    a.tdc = tdc;
    a.nt = til.nt;
    a.nper = nper;
    a.block = block;
    a.lds = til.lds_bytes;
    a.pb = til.pb;
    a.maxinc = til.maxinc;
    a.Eexp = Eexp;
    a.tiles = d_tiles;
    a.ent = d_ent;
    a.halo = d_halo;
    a.rec_of = d_rec_of;
    a.H = d_H;
    a.Tin = d_T[parity];
    a.Tout = d_T[1 - parity];
    a.loin = d_lo[parity];
    a.loout = d_lo[1 - parity];
    a.alpha = d_alpha;
    a.beta = d_beta;
    a.rA = d_rA;
    a.rAT = d_rAT;
    a.reA = d_reA;
    a.rTa = d_rTa;
    a.rP = d_rP;
    a.s0 = s0;
    a.s1 = s1;
    a.Tz = Tz;
    a.esk = d_esk;
    a.ktab = d_ktab;
    a.ctab = d_ctab;
    a.nkt = nkt;
    a.nct = nct;
    a.op = op;
    return a;
  }

  // the health check of a launch whose first step follows step count step0
  void health_args(fed::StepArgs &a, long long step0, bool energy) const {
    a.hl = d_health;
    a.hpart = d_hpart;
    a.win_lo = win_lo;
    a.win_hi = win_hi;
    // FP32 kernels compare in FP32: the window rounded outward, so no
    // temperature inside the FP64 window is flagged
    a.win_lo_f = (float)a.win_lo;
    a.win_hi_f = (float)a.win_hi;
    if ((double)a.win_lo_f > a.win_lo) a.win_lo_f = std::nextafter(a.win_lo_f, -INFINITY);
    if ((double)a.win_hi_f < a.win_hi) a.win_hi_f = std::nextafter(a.win_hi_f, INFINITY);
    a.step0 = step0;
    a.hbase = 0;
    a.energy = energy ? 1 : 0;
  }

  // record powers of step n (counted from fed_set_temperature) under the schedule
  const void *ps_row(int64_t n) const {
    return (const char *)d_psP + (size_t)rb * nrec * (size_t)(n % ps_rows);
  }

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    gsteps = 0;
    gparity = -1;
  }

  ~fed_ctx() {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    pool.free_all();
  }
};

namespace {

int save_checkpoint(fed_ctx *c, int64_t i, hipStream_t s);
int run_steps(fed_ctx *c, int64_t nsteps, hipStream_t s);
int seg_buffer(fed_ctx *c, int64_t g);

template <typename T>
hipError_t upload(DevPool &pool, T **d, const T *h, size_t n) {
  hipError_t e = pool.alloc((void **)d, n * sizeof(T));
  if (e != hipSuccess || n == 0) return e;
  return hipMemcpy(*d, h, n * sizeof(T), hipMemcpyHostToDevice);
}

bool finite(double v) { return std::isfinite(v); }

int validate(const fed_mesh *m, const fed_materials *mt, const fed_bcs *bc, const fed_options *o) {
  if (!m || !mt || !bc || !o) return fail(FED_E_ARG, "null argument");
  if (m->elem != FED_HEX8 && m->elem != FED_TET4) return fail(FED_E_ARG, "elem must be 4 or 8");
  if (m->n_nodes <= 0 || m->n_elems <= 0) return fail(FED_E_ARG, "empty mesh");
  if (m->n_nodes >= (1LL << 31) || m->n_elems >= (1LL << 31))
    return fail(FED_E_ARG, "mesh too large for 32-bit ids");
  if (!m->x || !m->y || !m->z || !m->conn) return fail(FED_E_ARG, "null mesh array");
  for (int64_t k = 0; k < m->n_nodes; k++)
    if (!finite(m->x[k]) || !finite(m->y[k]) || !finite(m->z[k]))
      return fail(FED_E_ARG, "non-finite coordinate at node %lld", (long long)k);
  const int64_t nc = (int64_t)m->elem * m->n_elems;
  for (int64_t i = 0; i < nc; i++)
    if (m->conn[i] < 0 || m->conn[i] >= m->n_nodes)
      return fail(FED_E_ARG, "connectivity entry %lld out of range", (long long)i);
  if (mt->n_materials < 1 || !mt->materials) return fail(FED_E_ARG, "no materials");
  for (int i = 0; i < mt->n_materials; i++) {
    const fed_material &q = mt->materials[i];
    if (!(q.rho > 0) || !finite(q.c0) || !finite(q.c1) || !finite(q.s0) || !finite(q.s1))
      return fail(FED_E_ARG, "material %d: rho must be positive and values finite", i);
    for (int r = 0; r < 6; r++)
      if (!finite(q.k[r])) return fail(FED_E_ARG, "material %d: non-finite k", i);
    if (mt->n_ktab && (q.s0 != 1.0 || q.s1 != 0.0))
      return fail(FED_E_ARG, "material %d: a k table needs s0 = 1 and s1 = 0", i);
    if (mt->n_ctab && q.c1 != 0.0)
      return fail(FED_E_ARG, "material %d: a c table needs c1 = 0", i);
    double clo = q.c0 + q.c1 * o->T_lo, chi = q.c0 + q.c1 * o->T_hi;
    double slo = q.s0 + q.s1 * o->T_lo, shi = q.s0 + q.s1 * o->T_hi;
    if (!(clo > 0 && chi > 0)) return fail(FED_E_ARG, "material %d: c(T) not positive on [T_lo, T_hi]", i);
    if (!(slo > 0 && shi > 0)) return fail(FED_E_ARG, "material %d: D(T) not positive on [T_lo, T_hi]", i);
  }
  for (int w = 0; w < 2; w++) {
    const int32_t n = w ? mt->n_ctab : mt->n_ktab;
    const double *tT = w ? mt->ctab_T : mt->ktab_T, *tf = w ? mt->ctab_f : mt->ktab_f;
    if (n == 0) continue;
    if (n < 2 || n > fed::kMaxTablePoints || !tT || !tf)
      return fail(FED_E_ARG, "%s table: need 2..%d points", w ? "c" : "k", fed::kMaxTablePoints);
    for (int i = 0; i < n; i++)
      if (!finite(tT[i]) || !(tf[i] > 0) || !finite(tf[i]) || (i && !(tT[i] > tT[i - 1])))
        return fail(FED_E_ARG, "%s table: T must increase strictly and f be positive and finite",
                    w ? "c" : "k");
  }
  if (mt->elem_material)
    for (int64_t e = 0; e < m->n_elems; e++)
      if (mt->elem_material[e] < 0 || mt->elem_material[e] >= mt->n_materials)
        return fail(FED_E_ARG, "elem_material[%lld] out of range", (long long)e);
  if (mt->elem_kscale)
    for (int64_t e = 0; e < m->n_elems; e++)
      if (!(mt->elem_kscale[e] > 0) || !finite(mt->elem_kscale[e]))
        return fail(FED_E_ARG, "elem_kscale[%lld] must be positive and finite", (long long)e);
  if (mt->elem_k)
    for (int64_t i = 0; i < 6 * m->n_elems; i++)
      if (!finite(mt->elem_k[i])) return fail(FED_E_ARG, "non-finite elem_k");
  if (bc->n_dir < 0 || (bc->n_dir > 0 && (!bc->dir_nodes || !bc->dir_T)))
    return fail(FED_E_ARG, "bad Dirichlet arrays");
  for (int64_t i = 0; i < bc->n_dir; i++)
    if (bc->dir_nodes[i] < 0 || bc->dir_nodes[i] >= m->n_nodes || !finite(bc->dir_T[i]))
      return fail(FED_E_ARG, "Dirichlet entry %lld invalid", (long long)i);
  if (bc->n_faces < 0) return fail(FED_E_ARG, "n_faces < 0");
  if (bc->n_faces > 0) {
    if (bc->face_nodes != 3 && bc->face_nodes != 4) return fail(FED_E_ARG, "face_nodes must be 3 or 4");
    if (!bc->faces) return fail(FED_E_ARG, "null faces");
    for (int64_t i = 0; i < bc->n_faces * bc->face_nodes; i++)
      if (bc->faces[i] < 0 || bc->faces[i] >= m->n_nodes)
        return fail(FED_E_ARG, "face entry %lld out of range", (long long)i);
    for (int64_t f = 0; f < bc->n_faces; f++) {
      if (bc->face_h && !(bc->face_h[f] >= 0 && finite(bc->face_h[f])))
        return fail(FED_E_ARG, "face_h[%lld] must be >= 0", (long long)f);
      if (bc->face_eps && !(bc->face_eps[f] >= 0 && bc->face_eps[f] <= 1))
        return fail(FED_E_ARG, "face_eps[%lld] must be in [0, 1]", (long long)f);
      if (bc->face_Ta && !finite(bc->face_Ta[f])) return fail(FED_E_ARG, "non-finite face_Ta");
      if (bc->face_q && !finite(bc->face_q[f])) return fail(FED_E_ARG, "non-finite face_q");
    }
  }
  if (bc->n_pt < 0 || (bc->n_pt > 0 && (!bc->pt_nodes || !bc->pt_W)))
    return fail(FED_E_ARG, "bad point-load arrays");
  for (int64_t i = 0; i < bc->n_pt; i++)
    if (bc->pt_nodes[i] < 0 || bc->pt_nodes[i] >= m->n_nodes || !finite(bc->pt_W[i]))
      return fail(FED_E_ARG, "point load %lld invalid", (long long)i);
  if (!finite(bc->Tz)) return fail(FED_E_ARG, "non-finite Tz");
  if (o->prec != FED_FP32C && o->prec != FED_FP64 && o->prec != FED_FP32)
    return fail(FED_E_ARG, "unknown precision %d", o->prec);
  if (!(o->dt >= 0) || !finite(o->dt)) return fail(FED_E_ARG, "dt must be >= 0");
  if (o->dt == 0 && !(o->safety > 0)) return fail(FED_E_ARG, "safety must be > 0 when dt == 0");
  if (!(o->T_hi > o->T_lo)) return fail(FED_E_ARG, "need T_lo < T_hi");
  if (o->node_instance)
    for (int64_t k = 0; k < m->n_nodes; k++)
      if (o->node_instance[k] < 0 || o->node_instance[k] >= m->n_nodes)
        return fail(FED_E_ARG, "node_instance[%lld] out of range", (long long)k);
  if (o->tile_nodes < 0) return fail(FED_E_ARG, "tile_nodes < 0");
  if (o->fuse_steps < 0 || o->fuse_steps > 4) return fail(FED_E_ARG, "fuse_steps must be in 0..4");
  if (o->block_threads != 0 &&
      (o->block_threads < 64 || o->block_threads > 1024 || o->block_threads % 64))
    return fail(FED_E_ARG, "block_threads must be a multiple of 64 in [64, 1024]");
  if (o->fuse_steps > 1 && o->block_threads > 512)
    return fail(FED_E_ARG, "block_threads must be <= 512 when fuse_steps > 1");
  if (o->resident != 0 && o->resident != 1) return fail(FED_E_ARG, "resident must be 0 or 1");
  if (o->resident && o->fuse_steps > 1) return fail(FED_E_ARG, "resident stepping needs fuse_steps <= 1");
  if (o->hex_gradient != 0 && o->hex_gradient != 1) return fail(FED_E_ARG, "hex_gradient must be 0 or 1");
  if (o->hex_gradient == 1 && m->elem == FED_HEX8 && o->fuse_steps > 1)
    return fail(FED_E_ARG, "the uniform-gradient hexahedron runs one step per launch or "
                           "resident (fuse_steps <= 1)");
  if (!(o->hourglass >= 0) || !std::isfinite(o->hourglass))
    return fail(FED_E_ARG, "hourglass must be a finite number >= 0");
  if (!(o->check_margin >= 0) || !std::isfinite(o->check_margin))
    return fail(FED_E_ARG, "check_margin must be a finite number >= 0");
  if (o->check_window != 0 && o->check_window != 1)
    return fail(FED_E_ARG, "check_window must be 0 or 1");
  if (o->check_every < 0) return fail(FED_E_ARG, "check_every must be >= 0");
  if (!(o->energy_tol >= 0) || !std::isfinite(o->energy_tol))
    return fail(FED_E_ARG, "energy_tol must be a finite number >= 0");
  if ((o->dev_alloc == nullptr) != (o->dev_free == nullptr))
    return fail(FED_E_ARG, "dev_alloc and dev_free must be given together");
  if (o->hourglass > 0 && !(m->elem == FED_HEX8 && o->hex_gradient == 1))
    return fail(FED_E_ARG, "hourglass control needs hexahedra with hex_gradient = 1");
  return FED_OK;
}

// Extreme of a piecewise-linear table (constant beyond its ends) on [lo, hi]:
// at the ends or at a breakpoint inside.
double table_extreme(const std::vector<double> &tT, const std::vector<double> &tf, double lo,
                     double hi, bool want_max) {
  const int n = (int)tT.size();
  auto at = [&](double T) {
    if (T <= tT[0]) return tf[0];
    if (T >= tT[n - 1]) return tf[n - 1];
    int i = 1;
    while (T > tT[i]) i++;
    return tf[i - 1] + (T - tT[i - 1]) / (tT[i] - tT[i - 1]) * (tf[i] - tf[i - 1]);
  };
  double r = want_max ? std::max(at(lo), at(hi)) : std::min(at(lo), at(hi));
  for (int i = 0; i < n; i++)
    if (tT[i] > lo && tT[i] < hi) r = want_max ? std::max(r, tf[i]) : std::min(r, tf[i]);
  return r;
}

// The stability bound (Sec. 3.4, Eq. 29) per instance for temperatures in
// [lo, hi], from the context's pre-computation (leaves the per-node minimum
// capacity of [lo, hi] in d_Cmin).
int bound_dt(fed_ctx *c, double lo, double hi, std::vector<double> &dtc, hipStream_t s) {
  const double fk = c->nkt ? table_extreme(c->h_ktab_T, c->h_ktab_f, lo, hi, true) : 1.0;
  const double fc = c->nct ? table_extreme(c->h_ctab_T, c->h_ctab_f, lo, hi, false) : 1.0;
  fed::MassArgs ma{c->N, c->ne, c->d_incp, c->d_ince, c->d_mats, c->d_emat, c->d_ec0, c->d_V,
                   lo, hi, c->d_M0, c->d_M1, c->d_Cmin, fc};
  HIPCHK(fed::launch_mass(ma, s));
  HIPCHK(hipMemsetAsync(c->d_lam, 0, sizeof(unsigned long long) * 2 * c->ninst, s));
  fed::DtArgs da{c->ne, c->E, c->nrec, c->d_lamgeo, c->d_kscale, c->d_mats, c->d_emat, c->d_ec0,
                 c->d_einst, c->d_recnode, c->d_ninst, c->d_b64[0], c->d_b64[2], c->d_Cmin,
                 lo, hi, c->Tz, c->d_lam, c->d_lam + c->ninst, fk, fc};
  HIPCHK(fed::launch_dt(da, s));
  std::vector<unsigned long long> lam(2 * c->ninst);
  HIPCHK(hipMemcpyAsync(lam.data(), c->d_lam, lam.size() * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  dtc.resize(c->ninst);
  for (int64_t i = 0; i < c->ninst; i++) {
    double le, lb;
    std::memcpy(&le, &lam[i], 8);
    std::memcpy(&lb, &lam[c->ninst + i], 8);
    dtc[i] = le + lb > 0 ? 2.0 / (le + lb) : INFINITY;
  }
  return FED_OK;
}

// The health window.  check_window 1: [T_lo - check_margin, T_hi +
// check_margin].  0: [T_lo - m, T_hi + m] with m the largest margin for which
// the time step in use stays within the stability bound over the window (the
// bound is derived for [T_lo, T_hi] and the step takes a safety factor below
// it, so the step stays provably stable a little beyond the range; m = 0 if
// the step exceeds the bound, unbounded where the bound does not depend on
// T).  Leaves d_Cmin as [T_lo, T_hi] gives it.
int derive_window(fed_ctx *c, hipStream_t s) {
  const double wlo0 = c->win_lo, whi0 = c->win_hi;
  if (c->check_window == 1) {
    c->win_lo = c->T_lo - c->check_margin;
    c->win_hi = c->T_hi + c->check_margin;
  } else {
    // margins that keep every law positive (c(T) > 0, s(T) > 0) on the window
    double cap = 1e6 * (1.0 + c->T_hi - c->T_lo);
    auto limit = [&](double a0, double a1) {  // a0 + a1 T > 0 on [T_lo - m, T_hi + m]
      if (a1 > 0) cap = std::min(cap, c->T_lo + a0 / a1);
      if (a1 < 0) cap = std::min(cap, -a0 / a1 - c->T_hi);
    };
    for (const fed_material &q : c->h_mats) {
      limit(q.c0, q.c1);
      limit(q.s0, q.s1);
    }
    cap = std::max(0.0, cap * (1.0 - 1e-9));
    std::vector<double> dtc;
    auto stable = [&](double m, bool &ok) -> int {
      int rc = bound_dt(c, c->T_lo - m, c->T_hi + m, dtc, s);
      if (rc) return rc;
      ok = true;
      for (int64_t i = 0; i < c->ninst; i++) ok &= c->dt_used[i] <= dtc[i];
      return FED_OK;
    };
    bool ok = false;
    int rc = stable(0.0, ok);
    if (rc) return rc;
    double m = 0.0;
    if (ok) {
      rc = stable(cap, ok);
      if (rc) return rc;
      if (ok) {
        m = cap >= 1e6 * (1.0 + c->T_hi - c->T_lo) * (1.0 - 1e-6) ? INFINITY : cap;
      } else {
        double a = 0.0, b = cap;  // stable at a, not at b
        for (int it = 0; it < 48 && b - a > 1e-9 * (1.0 + a); it++) {
          const double mid = 0.5 * (a + b);
          rc = stable(mid, ok);
          if (rc) return rc;
          (ok ? a : b) = mid;
        }
        m = a;
      }
    }
    c->win_lo = c->T_lo - m;
    c->win_hi = c->T_hi + m;
    std::vector<double> keep;
    rc = bound_dt(c, c->T_lo, c->T_hi, keep, s);  // d_Cmin of the range itself
    if (rc) return rc;
  }
  // captured graph launches carry the window
  if (c->win_lo != wlo0 || c->win_hi != whi0) c->drop_graph();
  return FED_OK;
}

// Exported nodes and exchange buffers of resident stepping; checks that every
// tile fits the kernel's registers and that all tiles are resident at once.
// *exch receives the bytes one step moves through memory.
int setup_resident(fed_ctx *c, int n_cu, double *exch) {
  const fed::Tiling &T = c->til;
  const int64_t N = c->N;
  const fed::ResCaps cap = fed::resident_caps(c->prec, c->ne);
  for (int32_t t = 0; t < T.nt; t++) {
    const fed::TileHdr &th = T.tiles[t];
    const int nE = th.cum_e[0], nhalo = th.cum_n[1] - th.nown;
    if (th.nown > cap.npt * c->block || nE > cap.ept * c->block || nhalo > cap.hpt * c->block)
      return fail(FED_E_MESH,
                  "resident stepping: tile %d (%d nodes, %d elements, %d halo nodes) exceeds the "
                  "%d threads' registers (%d / %d / %d per thread); use more tiles or resident = 0",
                  t, th.nown, nE, nhalo, c->block, cap.npt, cap.ept, cap.hpt);
  }
  // Overlapping the tile-interior elements with the halo wait costs a third
  // workgroup barrier a step; it pays unless the element work is long enough
  // to cover the exchange anyway, as with tables or per-element laws (64^3
  // hexahedra with the linear laws: 2.37 against 2.67 us FP32C, 3.15 against
  // 3.36 us FP64; with tables: 4.08 against 3.89 us FP32C, 4.91 against 4.76
  // us FP64)
  c->res_split = (c->d_esk || c->d_ktab || c->d_ctab) ? 0 : 1;
  std::vector<uint8_t> exported(N, 0);
  int64_t halo_total = 0;
  for (int32_t t = 0; t < T.nt; t++) {
    const fed::TileHdr &th = T.tiles[t];
    const int nhalo = th.cum_n[1] - th.nown;
    halo_total += nhalo;
    for (int j = 0; j < nhalo; j++) exported[T.halo[th.hstart + j]] = 1;
  }
  DevPool &P = c->pool;
  HIPCHK(upload(P, &c->d_exported, exported.data(), exported.size()));
  // FP32 hexahedra with the folded operator and the shared laws: each tile's
  // touched nodes take LDS positions in caller order, so the temperatures
  // and slots a wave's elements touch are mostly consecutive words (the
  // tile's own order groups its nodes by the tiles that read them)
  c->res_sstride = 0;
  if (c->ne == FED_HEX8 && c->op == 0 && c->rb == 4 && !(c->d_ktab || c->d_ctab || c->d_esk)) {
    std::vector<int16_t> sigma;
    std::vector<uint16_t> ents;
    int32_t stride = 0;
    if (fed::caller_order_positions(T, c->ne, sigma, stride, ents)) {
      HIPCHK(upload(P, &c->d_sigma, sigma.data(), sigma.size()));
      HIPCHK(upload(P, &c->d_ent_sigma, ents.data(), ents.size()));
      c->res_sstride = stride;
    }
  }
  const int words = c->prec == FED_FP64 ? 2 : 1;
  for (int i = 0; i < 2; i++) {
    HIPCHK(P.alloc((void **)&c->d_X[i], sizeof(unsigned long long) * words * N));
    HIPCHK(hipMemset(c->d_X[i], 0, sizeof(unsigned long long) * words * N));  // tag 0: never wanted
  }
  HIPCHK(P.alloc((void **)&c->d_rerr, sizeof(int)));
  HIPCHK(hipMemset(c->d_rerr, 0, sizeof(int)));
  // LDS of the resident kernel: T of the touched nodes, the slots of the
  // touched nodes (hexahedra, except the FP32 uniform-gradient instance that
  // keeps halo elements' operators, and in FP64 the uniform-gradient one and
  // the general laws: 2^pb + 1 each) or of the owned nodes (the others: maxinc
  // each), the 5 boundary coefficients of the owned boundary nodes and, with a
  // conductivity table where every tile has room for it, the table's value at
  // every touched node (else the elements evaluate it at their nodes)
  // (the FP32 uniform-gradient hexahedron without hourglass control and with
  // the shared laws adds, where every tile has room for them, the operators
  // of its elements that touch the halo)
  const bool gen = c->d_ktab || c->d_ctab || c->d_esk;  // the kernel's general-law instance
  const bool oph_inst = c->op == 1 && !gen && c->rb == 4;  // the kernel's OPH instances
  const bool nm = c->ne == FED_HEX8 && (c->op == 0 || (c->rb == 4 && !oph_inst)) &&
                  !(gen && c->rb == 8);
  auto need = [&](bool nv, bool oph) {
    int64_t m = 0;
    for (const fed::TileHdr &th : T.tiles) {
      const int64_t ns = nm ? (int64_t)th.cum_n[1] * ((1 << T.pb) + 1) : (int64_t)T.maxinc * th.nown;
      const int64_t nh = th.cum_e[0] - (c->res_split ? th.nint : 0);  // elements after the wait
      m = std::max<int64_t>(m, (int64_t)c->rb * (th.cum_n[1] + ns + 5LL * th.nbnd +
                                                  (nv ? th.cum_n[1] : 0) +
                                                  (oph ? (int64_t)(c->hw | 1) * nh : 0)) +
                                   16);
    }
    return m;
  };
  const int64_t lds_limit = c->max_lds - kStaticLds;
  c->res_nv = c->nkt > 0 && need(true, false) <= lds_limit;
  c->res_oph = oph_inst && need(c->res_nv, true) <= lds_limit;
  const int64_t lds = need(c->res_nv, c->res_oph);
  c->res_oph_elems = 0;
  if (c->res_oph)
    for (const fed::TileHdr &th : T.tiles) c->res_oph_elems += th.cum_e[0] - (c->res_split ? th.nint : 0);
  if (lds > c->max_lds - kStaticLds)
    return fail(FED_E_MESH, "resident stepping: a tile needs %lld bytes of LDS (the GPU has %d, "
                "%d of them taken by the health check)",
                (long long)lds, c->max_lds, kStaticLds);
  c->res_lds = (int)lds;
  int per_cu = 0;
  fed::StepArgs a0 = c->step_args(0, 1);
  a0.lds = c->res_lds;
  HIPCHK(fed::resident_prepare(a0, &per_cu));
  const int64_t grid = 8LL * c->nper;
  if (per_cu < 1 || grid > (int64_t)per_cu * n_cu)
    return fail(FED_E_MESH,
                "resident stepping: %lld workgroups of %d threads and %d bytes of LDS, but the GPU "
                "holds %d at once (%d per CU); use larger tiles, fewer threads or resident = 0",
                (long long)grid, c->block, c->res_lds, per_cu * n_cu, per_cu);
  int64_t nexp = 0;
  for (uint8_t v : exported) nexp += v;
  *exch = 8.0 * words * (double)(halo_total + nexp);  // tagged words read and written
  // resident adjoint: the FP64 boundary sums (and, in FP64, the elements'
  // derivative sums and rho V / n_e); mu, w, T^n, T^{n+1}, alpha, 1/dt (and beta) and
  // the node-major slots of the touched nodes, hA and sigma eps A of the
  // owned boundary nodes; offered where it fits, else fed_backward runs one
  // adjoint step per launch
  // (per-element laws run the one-step adjoint, which reads them)
  if (c->ne == FED_HEX8 && c->op == 0 && !c->d_esk) {
    int64_t alds = 0;
    for (const fed::TileHdr &th : T.tiles)
      alds = std::max<int64_t>(alds, 16LL * th.nbnd + (c->prec == FED_FP64 ? 24LL * th.cum_e[0] : 0) +
                                         (int64_t)c->rb * ((6 + (c->tdc ? 1 : 0) + (1 << T.pb) + 1) *
                                                               (int64_t)th.cum_n[1] + 2LL * th.nbnd) + 16);
    int aper = 0;
    if (alds <= c->max_lds) {
      HIPCHK(fed::adjres_prepare(c->prec == FED_FP64 ? 1 : (c->prec == FED_FP32C ? 0 : 2),
                                 c->d_ktab || c->d_ctab || c->d_esk, c->block,
                                 (int)alds, &aper));
      if (aper >= 1 && grid <= (int64_t)aper * n_cu) {
        c->adjres = true;
        c->adjres_lds = (int)alds;
      }
    }
  }
  return FED_OK;
}

}  // namespace

extern "C" {

const char *fed_last_error(void) { return g_err.c_str(); }

int fed_create(const fed_mesh *m, const fed_materials *mt, const fed_bcs *bc,
               const fed_options *o, void *stream, fed_ctx **out) {
  if (!out) return fail(FED_E_ARG, "null out");
  *out = nullptr;
  int rc = validate(m, mt, bc, o);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = m->n_nodes, E = m->n_elems;
  const int ne = m->elem;
  std::unique_ptr<fed_ctx> c(new (std::nothrow) fed_ctx());
  if (!c) return fail(FED_E_NOMEM, "host allocation failed");
  c->prec = o->prec;
  c->pool.af = o->dev_alloc;
  c->pool.ff = o->dev_free;
  c->pool.actx = o->alloc_ctx;
  c->ne = ne;
  c->rb = o->prec == FED_FP64 ? 8 : 4;
  c->N = N;
  c->E = E;
  c->Tz = bc->Tz;
  c->T_lo = o->T_lo;
  c->T_hi = o->T_hi;
  c->s0 = mt->materials[0].s0;
  c->s1 = mt->materials[0].s1;
  bool mixed_k = false;
  for (int i = 0; i < mt->n_materials; i++) {
    c->tdk |= mt->materials[i].s1 != 0.0;
    c->tdc |= mt->materials[i].c1 != 0.0;
    mixed_k |= mt->materials[i].s0 != c->s0 || mt->materials[i].s1 != c->s1;
  }
  c->tdk |= mt->n_ktab > 0;
  c->tdc |= mt->n_ctab > 0;
  c->nkt = mt->n_ktab;
  c->nct = mt->n_ctab;
  c->h_mats.assign(mt->materials, mt->materials + mt->n_materials);
  if (c->nkt) {
    c->h_ktab_T.assign(mt->ktab_T, mt->ktab_T + c->nkt);
    c->h_ktab_f.assign(mt->ktab_f, mt->ktab_f + c->nkt);
    c->fk_max = table_extreme(c->h_ktab_T, c->h_ktab_f, o->T_lo, o->T_hi, true);
  }
  if (c->nct) {
    c->h_ctab_T.assign(mt->ctab_T, mt->ctab_T + c->nct);
    c->h_ctab_f.assign(mt->ctab_f, mt->ctab_f + c->nct);
    c->fc_min = table_extreme(c->h_ctab_T, c->h_ctab_f, o->T_lo, o->T_hi, false);
  }
  c->resident = o->resident == 1;
  c->op = (ne == FED_HEX8 && o->hex_gradient == 1) ? (o->hourglass > 0 ? 2 : 1) : 0;
  c->hw = c->op == 2 ? 40 : c->op ? 27 : 6;
  c->hg_eps = c->op == 2 ? o->hourglass : 0.0;
  c->block = o->block_threads ? o->block_threads : (c->resident ? 1024 : 256);

  // ---- host index work: boundary records, instances, tiling ---------------
  std::vector<uint8_t> has_bnd(N, 0);
  for (int64_t i = 0; i < bc->n_faces * bc->face_nodes; i++) has_bnd[bc->faces[i]] = 1;
  for (int64_t i = 0; i < bc->n_pt; i++) has_bnd[bc->pt_nodes[i]] = 1;
  // radiation ambient must be single-valued per node
  std::vector<double> taR(N, 0.0);
  std::vector<uint8_t> taSet(N, 0);
  for (int64_t f = 0; f < bc->n_faces; f++) {
    double eps = bc->face_eps ? bc->face_eps[f] : 0.0;
    if (eps <= 0) continue;
    double ta = bc->face_Ta ? bc->face_Ta[f] : 0.0;
    for (int b = 0; b < bc->face_nodes; b++) {
      int32_t k = bc->faces[f * bc->face_nodes + b];
      if (taSet[k] && taR[k] != ta)
        return fail(FED_E_ARG, "radiating faces at node %d have different Ta", k);
      taSet[k] = 1;
      taR[k] = ta;
    }
  }
  c->ninst = 1;
  if (o->node_instance) {
    int32_t mx = 0;
    for (int64_t k = 0; k < N; k++) mx = std::max(mx, o->node_instance[k]);
    c->ninst = (int64_t)mx + 1;
    for (int64_t e = 0; e < E; e++)
      for (int a = 1; a < ne; a++)
        if (o->node_instance[m->conn[(int64_t)a * E + e]] != o->node_instance[m->conn[e]])
          return fail(FED_E_ARG, "element %lld spans two instances", (long long)e);
  }
  int dev = 0, n_cu = 1, max_lds = 64 * 1024;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  c->max_lds = max_lds;
  fed::TilingInput ti;
  ti.N = N;
  ti.E = E;
  ti.ne = ne;
  ti.x = m->x;
  ti.y = m->y;
  ti.z = m->z;
  ti.conn = m->conn;
  ti.node_instance = o->node_instance;
  ti.has_bnd = has_bnd.data();
  ti.target_nodes = o->tile_nodes ? o->tile_nodes : 512;
  ti.depth = o->fuse_steps ? o->fuse_steps : 1;
  ti.lds_budget = 64 * 1024;
  ti.real_bytes = c->rb;
  // staged per updated node: alpha, beta, record id, and lo for FP32C
  ti.upd_bytes = 2 * c->rb + 4 + (c->prec == FED_FP32C ? 4 : 0);
  // a conductivity table's value at every touched node, staged with its T
  ti.touch_bytes = c->nkt > 0 ? c->rb : 0;
  // resident stepping: one workgroup per CU for every 1024 threads a CU holds,
  // tiles as large as the node count over that many workgroups; only T of the
  // touched nodes and the slots live in LDS
  const int res_per_cu = std::max(1, 1024 / c->block);
  if (c->resident) {
    const int64_t wgs = (int64_t)n_cu * res_per_cu;
    if (!o->tile_nodes) ti.target_nodes = (int32_t)std::max<int64_t>(1, (N + wgs - 1) / wgs);
    ti.depth = 1;
    ti.lds_budget = max_lds - kStaticLds;
    ti.upd_bytes = 0;
  }
  std::string terr;
  for (int attempt = 0;; attempt++) {
    terr = fed::build_tiling(ti, c->til);
    if (!terr.empty() || !c->resident || o->tile_nodes) break;
    // resident: grow the tiles until the grid (tiles rounded up to whole XCD
    // rounds) fits the resident workgroups; instances split separately can
    // leave more tiles than the node count over the tile size
    const int64_t wgs = (int64_t)n_cu * res_per_cu, grid = 8LL * ((c->til.nt + 7) / 8);
    if (grid <= wgs || attempt >= 8) break;
    ti.target_nodes = (int32_t)std::min<double>(1e9, ti.target_nodes * 1.05 * (double)grid / wgs + 1);
  }
  if (!terr.empty()) return fail(FED_E_MESH, "tiling: %s", terr.c_str());
  fed::Tiling &T = c->til;
  c->Eexp = (int64_t)T.eorig.size();
  c->nper = (T.nt + 7) / 8;
  c->K = T.depth;
  // boundary records in internal order + their (face | point) items
  std::vector<int32_t> rec_node;
  std::vector<std::vector<int32_t>> items_of(N);
  for (int64_t f = 0; f < bc->n_faces; f++)
    for (int b = 0; b < bc->face_nodes; b++) items_of[bc->faces[f * bc->face_nodes + b]].push_back((int32_t)f);
  for (int64_t i = 0; i < bc->n_pt; i++) items_of[bc->pt_nodes[i]].push_back(-(int32_t)(i + 1));
  std::vector<int64_t> rec_ptr{0};
  std::vector<int32_t> rec_item;
  std::vector<double> rec_ta;
  for (int32_t t = 0; t < T.nt; t++) {
    const fed::TileHdr &th = T.tiles[t];
    for (int32_t j = 0; j < th.nbnd; j++) {
      int32_t ki = th.nstart + j, k = T.iperm[ki];
      rec_node.push_back(ki);
      for (int32_t it : items_of[k]) rec_item.push_back(it);
      rec_ptr.push_back((int64_t)rec_item.size());
      rec_ta.push_back(taR[k]);
    }
  }
  items_of.clear();
  items_of.shrink_to_fit();
  c->nrec = (int64_t)rec_node.size();
  std::vector<int32_t> rec_of(N, -1);
  for (size_t r = 0; r < rec_node.size(); r++) rec_of[rec_node[r]] = (int32_t)r;
  std::vector<int32_t> node_inst_int, elem_inst;
  if (o->node_instance) {
    node_inst_int.resize(N);
    for (int64_t k = 0; k < N; k++) node_inst_int[T.perm[k]] = o->node_instance[k];
    elem_inst.resize(E);
    for (int64_t e = 0; e < E; e++) elem_inst[e] = o->node_instance[m->conn[e]];
  }
  std::vector<uint8_t> is_dir(N, 0);
  std::vector<int32_t> dir_node(bc->n_dir);
  for (int64_t i = 0; i < bc->n_dir; i++) {
    dir_node[i] = T.perm[bc->dir_nodes[i]];
    is_dir[dir_node[i]] = 1;
  }
  c->ndir = bc->n_dir;

  // ---- device pre-computation in FP64 (Sec. 3.5 (i)) ------------------------
  DevPool tmp;
  tmp.af = o->dev_alloc;
  tmp.ff = o->dev_free;
  tmp.actx = o->alloc_ctx;
  struct TmpGuard {
    DevPool &p;
    ~TmpGuard() { p.free_all(); }
  } guard{tmp};
  DevPool &P = c->pool;
  double *d_x, *d_y, *d_z;
  int32_t *d_conn;
  fed::MatDev *d_mats;
  int32_t *d_emat = nullptr;
  double *d_ek = nullptr;
  HIPCHK(upload(tmp, &d_x, m->x, N));
  HIPCHK(upload(tmp, &d_y, m->y, N));
  HIPCHK(upload(tmp, &d_z, m->z, N));
  HIPCHK(upload(tmp, &d_conn, m->conn, (size_t)ne * E));
  static_assert(sizeof(fed::MatDev) == sizeof(fed_material), "material layout");
  HIPCHK(upload(P, &d_mats, reinterpret_cast<const fed::MatDev *>(mt->materials),
                (size_t)mt->n_materials));
  if (mt->elem_material) HIPCHK(upload(P, &d_emat, mt->elem_material, (size_t)E));
  c->d_mats = d_mats;
  c->d_emat = d_emat;
  if (mt->elem_k) HIPCHK(upload(tmp, &d_ek, mt->elem_k, (size_t)6 * E));
  {
    std::vector<double> ks(E, 1.0);
    if (mt->elem_kscale) std::copy(mt->elem_kscale, mt->elem_kscale + E, ks.begin());
    HIPCHK(upload(P, &c->d_kscale, ks.data(), (size_t)E));
  }
  int *d_cnt;
  HIPCHK(tmp.alloc((void **)&d_cnt, 2 * sizeof(int)));
  HIPCHK(hipMemsetAsync(d_cnt, 0, 2 * sizeof(int), s));
  double *d_lamgeo;
  HIPCHK(P.alloc((void **)&c->d_H0, sizeof(double) * c->hw * E));
  HIPCHK(P.alloc((void **)&c->d_V, sizeof(double) * E));
  HIPCHK(P.alloc((void **)&d_lamgeo, sizeof(double) * E));
  c->d_lamgeo = d_lamgeo;
  fed::GeomArgs ga{ne, E, d_x, d_y, d_z, d_conn, d_mats, d_emat, d_ek,
                   c->d_H0, c->op, c->d_V, d_lamgeo, d_cnt, d_cnt + 1, c->hg_eps};
  HIPCHK(fed::launch_geom(ga, s));
  int cnt[2];
  HIPCHK(hipMemcpyAsync(cnt, d_cnt, sizeof(cnt), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (cnt[0]) return fail(FED_E_MESH, "%d inverted or degenerate elements", cnt[0]);
  if (cnt[1]) return fail(FED_E_ARG, "%d conductivity tensors are not positive definite", cnt[1]);
  // lumped capacity per internal node
  int64_t *d_incp;
  int32_t *d_ince;
  HIPCHK(upload(P, &d_incp, T.inc_ptr.data(), T.inc_ptr.size()));
  HIPCHK(upload(P, &d_ince, T.inc_elem.data(), T.inc_elem.size()));
  c->d_incp = d_incp;
  c->d_ince = d_ince;
  double *d_Cmin;
  HIPCHK(P.alloc((void **)&c->d_M0, sizeof(double) * N));
  HIPCHK(P.alloc((void **)&c->d_M1, sizeof(double) * N));
  HIPCHK(P.alloc((void **)&d_Cmin, sizeof(double) * N));
  c->d_Cmin = d_Cmin;
  fed::MassArgs ma{N, ne, d_incp, d_ince, d_mats, d_emat, nullptr, c->d_V, o->T_lo, o->T_hi,
                   c->d_M0, c->d_M1, d_Cmin, c->fc_min};
  HIPCHK(fed::launch_mass(ma, s));
  // boundary lumping
  int32_t *d_faces = nullptr, *d_recitem = nullptr, *d_recnode = nullptr;
  int64_t *d_recptr = nullptr;
  double *d_fh = nullptr, *d_fTa = nullptr, *d_feps = nullptr, *d_fq = nullptr, *d_farea = nullptr;
  double *d_ptW = nullptr, *b64[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const int64_t nf = bc->n_faces;
  c->nf = nf;
  c->nfn = bc->face_nodes;
  if (nf > 0) {
    // every face array exists on the device (zeros for NULL) so that
    // fed_set_params can replace h later
    std::vector<double> zeros(nf, 0.0);
    HIPCHK(upload(P, &d_faces, bc->faces, (size_t)nf * bc->face_nodes));
    HIPCHK(upload(P, &d_fh, bc->face_h ? bc->face_h : zeros.data(), (size_t)nf));
    HIPCHK(upload(P, &d_fTa, bc->face_Ta ? bc->face_Ta : zeros.data(), (size_t)nf));
    HIPCHK(upload(P, &d_feps, bc->face_eps ? bc->face_eps : zeros.data(), (size_t)nf));
    HIPCHK(upload(P, &d_fq, bc->face_q ? bc->face_q : zeros.data(), (size_t)nf));
    HIPCHK(P.alloc((void **)&d_farea, sizeof(double) * nf));
    if (bc->face_eps)
      for (int64_t f = 0; f < nf; f++) c->has_rad |= bc->face_eps[f] > 0;
    c->h_faces.assign(bc->faces, bc->faces + (size_t)nf * bc->face_nodes);
    c->h_feps.assign(nf, 0.0);
    if (bc->face_eps) c->h_feps.assign(bc->face_eps, bc->face_eps + nf);
  }
  c->npt = bc->n_pt;
  if (bc->n_pt > 0) HIPCHK(upload(P, &d_ptW, bc->pt_W, (size_t)bc->n_pt));
  const int64_t nrec = c->nrec;
  if (nrec > 0) {
    HIPCHK(upload(P, &d_recptr, rec_ptr.data(), rec_ptr.size()));
    HIPCHK(upload(P, &d_recitem, rec_item.data(), rec_item.size()));
    HIPCHK(upload(P, &d_recnode, rec_node.data(), rec_node.size()));
    for (int i = 0; i < 4; i++) HIPCHK(P.alloc((void **)&b64[i], sizeof(double) * nrec));
    HIPCHK(upload(P, &b64[4], rec_ta.data(), rec_ta.size()));
  }
  c->d_faces = d_faces;
  c->d_fh = d_fh;
  c->d_fTa = d_fTa;
  c->d_feps = d_feps;
  c->d_fq = d_fq;
  c->d_farea = d_farea;
  c->d_ptW = d_ptW;
  c->d_recptr = d_recptr;
  c->d_recitem = d_recitem;
  c->d_recnode = d_recnode;
  for (int i = 0; i < 5; i++) c->d_b64[i] = b64[i];
  fed::BndArgs ba{nf, bc->face_nodes, d_faces, d_x, d_y, d_z, d_fh, d_fTa, d_feps, d_fq,
                  d_farea, nrec, d_recptr, d_recitem, d_ptW, b64[0], b64[1], b64[2], b64[3],
                  nullptr};
  HIPCHK(fed::launch_bnd(ba, s));
  // stability bound per instance (Sec. 3.4)
  int32_t *d_einst = nullptr, *d_ninst = nullptr;
  if (o->node_instance) {
    HIPCHK(upload(P, &d_einst, elem_inst.data(), elem_inst.size()));
    HIPCHK(upload(P, &d_ninst, node_inst_int.data(), node_inst_int.size()));
  }
  c->d_einst = d_einst;
  c->d_ninst = d_ninst;
  c->allow_unstable = o->allow_unstable != 0;
  unsigned long long *d_lam;
  HIPCHK(P.alloc((void **)&d_lam, sizeof(unsigned long long) * 2 * c->ninst));
  c->d_lam = d_lam;
  HIPCHK(hipMemsetAsync(d_lam, 0, sizeof(unsigned long long) * 2 * c->ninst, s));
  fed::DtArgs da{ne, E, nrec, d_lamgeo, c->d_kscale, d_mats, d_emat, nullptr, d_einst, d_recnode,
                 d_ninst, b64[0], b64[2], d_Cmin, o->T_lo, o->T_hi, bc->Tz, d_lam,
                 d_lam + c->ninst, c->fk_max, c->fc_min};
  HIPCHK(fed::launch_dt(da, s));
  std::vector<unsigned long long> lam(2 * c->ninst);
  HIPCHK(hipMemcpyAsync(lam.data(), d_lam, lam.size() * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  c->dt_crit.resize(c->ninst);
  c->dt_used.resize(c->ninst);
  for (int64_t i = 0; i < c->ninst; i++) {
    double le, lb;
    std::memcpy(&le, &lam[i], 8);
    std::memcpy(&lb, &lam[c->ninst + i], 8);
    double l = le + lb;
    c->dt_crit[i] = l > 0 ? 2.0 / l : INFINITY;
    if (o->dt > 0) {
      c->dt_used[i] = o->dt;
      if (o->dt > c->dt_crit[i] && !o->allow_unstable)
        return fail(FED_E_UNSTABLE, "dt %.6g exceeds dt_crit %.6g (instance %lld)", o->dt,
                    c->dt_crit[i], (long long)i);
    } else {
      if (!std::isfinite(c->dt_crit[i]))
        return fail(FED_E_ARG, "dt_crit is unbounded (no conduction or boundary exchange); give dt");
      c->dt_used[i] = o->safety * c->dt_crit[i];
    }
  }
  c->check_margin = o->check_margin;
  c->check_window = o->check_window;
  rc = derive_window(c.get(), s);
  if (rc) return rc;
  // ---- working arrays in the step precision ---------------------------------
  const int rb = c->rb;
  double *d_dtinst;
  uint8_t *d_isdir;
  HIPCHK(upload(P, &d_dtinst, c->dt_used.data(), c->dt_used.size()));
  HIPCHK(upload(P, &d_isdir, is_dir.data(), is_dir.size()));
  c->d_dtinst = d_dtinst;
  c->d_isdir = d_isdir;
  HIPCHK(P.alloc(&c->d_alpha, (size_t)rb * N));
  if (c->tdc) HIPCHK(P.alloc(&c->d_beta, (size_t)rb * N));
  else {
    HIPCHK(P.alloc(&c->d_beta, (size_t)rb * N));
  }
  void **recs[5] = {&c->d_rA, &c->d_rAT, &c->d_reA, &c->d_rTa, &c->d_rP};
  for (int i = 0; i < 5; i++) HIPCHK(P.alloc(recs[i], (size_t)rb * std::max<int64_t>(nrec, 1)));
  fed::NodeArrArgs na{c->prec, N, nrec, c->d_M0, c->d_M1, d_dtinst, d_ninst, d_isdir,
                      b64[0], b64[1], b64[2], b64[4], b64[3],
                      c->d_alpha, c->d_beta, c->d_rA, c->d_rAT, c->d_reA, c->d_rTa, c->d_rP};
  HIPCHK(fed::launch_node_arrays(na, s));
  HIPCHK(upload(P, &c->d_eorig, T.eorig.data(), T.eorig.size()));
  HIPCHK(upload(P, &c->d_eowner, T.eowner.data(), T.eowner.size()));
  HIPCHK(P.alloc(&c->d_H, (size_t)rb * c->hw * c->Eexp));
  HIPCHK(fed::launch_expand_H(c->prec == FED_FP64 ? 1 : 0, c->hw, c->hs_from(), c->hs_to(), c->Eexp, E,
                              c->d_eorig, c->d_H0,
                              c->d_kscale, c->d_H, s));
  if (mixed_k) {
    HIPCHK(P.alloc(&c->d_esk, (size_t)rb * 2 * c->Eexp));
    HIPCHK(fed::launch_expand_sk(c->prec == FED_FP64 ? 1 : 0, c->Eexp, c->d_eorig, d_mats, d_emat,
                                 c->d_esk, s));
  }
  for (int w = 0; w < 2; w++) {
    const int32_t n = w ? c->nct : c->nkt;
    if (!n) continue;
    const double *tT = w ? mt->ctab_T : mt->ktab_T, *tf = w ? mt->ctab_f : mt->ktab_f;
    void **dst = w ? &c->d_ctab : &c->d_ktab;
    if (rb == 8) {
      std::vector<double> v(tT, tT + n);
      v.insert(v.end(), tf, tf + n);
      HIPCHK(upload(P, (double **)dst, v.data(), v.size()));
    } else {
      std::vector<float> v;
      for (int i = 0; i < n; i++) v.push_back((float)tT[i]);
      for (int i = 0; i < n; i++) v.push_back((float)tf[i]);
      HIPCHK(upload(P, (float **)dst, v.data(), v.size()));
    }
  }
  HIPCHK(upload(P, &c->d_tiles, T.tiles.data(), T.tiles.size()));
  HIPCHK(upload(P, &c->d_ent, T.ent.data(), T.ent.size()));
  if (T.halo.empty()) T.halo.push_back(0);  // keep a valid (unused) device array
  HIPCHK(upload(P, &c->d_halo, T.halo.data(), T.halo.size()));
  HIPCHK(upload(P, &c->d_perm, T.perm.data(), T.perm.size()));
  HIPCHK(upload(P, &c->d_rec_of, rec_of.data(), rec_of.size()));
  HIPCHK(P.alloc(&c->d_T[0], (size_t)rb * N));
  HIPCHK(P.alloc(&c->d_T[1], (size_t)rb * N));
  if (c->prec == FED_FP32C) {
    HIPCHK(P.alloc((void **)&c->d_lo[0], sizeof(float) * N));
    HIPCHK(P.alloc((void **)&c->d_lo[1], sizeof(float) * N));
  }
  if (c->ndir) {
    HIPCHK(upload(P, &c->d_dir_node, dir_node.data(), dir_node.size()));
    HIPCHK(upload(P, &c->d_dir_T, bc->dir_T, (size_t)c->ndir));
  }
  HIPCHK(P.alloc((void **)&c->d_health, sizeof(fed::Health)));
  HIPCHK(P.alloc((void **)&c->d_hpart, sizeof(double) * 2 * std::max(T.nt, 1)));
  HIPCHK(fed::launch_health(c->d_health, 0, 0, s));
  c->check_every = o->check_every;
  c->energy_tol = o->energy_tol;
  HIPCHK(P.alloc((void **)&c->d_flag, sizeof(int)));
  HIPCHK(P.alloc((void **)&c->d_rkeys, 2 * sizeof(unsigned long long)));
  HIPCHK(P.alloc((void **)&c->d_rnan, sizeof(int)));
  HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
  HIPCHK(P.alloc((void **)&c->d_Tuser, sizeof(double) * N));
  if (T.lds_bytes > max_lds)
    return fail(FED_E_MESH, "tile needs %d bytes of LDS", T.lds_bytes);
  HIPCHK(fed::step_set_lds_limit(c->prec == FED_FP64 ? 1 : (c->prec == FED_FP32C ? 0 : 2), ne,
                                 c->tdk, c->tdc, c->d_esk || c->d_ktab || c->d_ctab, c->op,
                                 std::max(T.lds_bytes, 1)));
  // LDS of the adjoint step: mu, T^n and the scaled increment of the touched
  // nodes of the first ring, and the slots of the owned nodes
  for (const fed::TileHdr &th : T.tiles)
    c->adj_lds = std::max(c->adj_lds, rb * (3 * th.cum_n[1] + T.maxinc * th.nown));
  if (c->adj_lds <= max_lds)
    HIPCHK(fed::adjoint_set_lds_limit(c->prec, ne, c->op, std::max(c->adj_lds, 1)));
  double exch_bytes = 0;
  if (c->resident) {
    int rc2 = setup_resident(c.get(), n_cu, &exch_bytes);
    if (rc2) return rc2;
  }
  HIPCHK(hipStreamSynchronize(s));
  // ---- info -------------------------------------------------------------------
  fed_info &I = c->info;
  I.n_nodes = N;
  I.n_elems = E;
  I.n_instances = c->ninst;
  I.n_tiles = T.nt;
  I.n_elems_expanded = c->Eexp;
  int64_t nhalo = 0;
  for (const fed::TileHdr &th : T.tiles) nhalo += th.nhalo;
  I.n_halo = nhalo;
  I.n_bnd_nodes = nrec;
  I.elem = ne;
  I.prec = c->prec;
  I.block_threads = c->block;
  I.lds_bytes = T.lds_bytes;
  // unique bytes of one launch (which advances K steps): per element its packed
  // entries (2 B / node) and the 6-entry operator; per node T read + write (and
  // lo read + write for FP32C), alpha (and beta when c depends on T); per
  // boundary node its 5 coefficients.  "Moved" counts what the launch requests:
  // every tile's copy of its elements, T (and lo) of its halo, the halo ids, the
  // coefficients of every node it updates, and the tile headers.
  I.fuse_steps = T.depth;
  I.resident = c->resident ? 1 : 0;
  I.exchange_bytes_per_step = exch_bytes;
  I.resident_adjoint = c->adjres ? 1 : 0;
  double elem_b = 2.0 * ne + c->hw * rb + (c->d_esk ? 2.0 * rb : 0.0);
  double lo_b = c->prec == FED_FP32C ? 4.0 : 0.0;
  double coef_b = rb + (c->tdc ? rb : 0.0);
  double node_b = 2.0 * rb + 2.0 * lo_b + coef_b;
  I.algorithmic_bytes_per_launch = elem_b * E + node_b * N + 5.0 * rb * nrec;
  double moved = elem_b * c->Eexp + sizeof(fed::TileHdr) * T.nt;
  for (const fed::TileHdr &th : T.tiles) {
    int64_t nupd = th.cum_n[T.depth - 1], ntouch = th.cum_n[T.depth];
    moved += (rb + 4.0) * (ntouch - th.nown) + rb * th.nown;   // T reads (+ halo ids)
    moved += (lo_b + coef_b) * nupd + 4.0 * (nupd - th.nown);  // lo, coefficients, rec ids
    moved += (rb + lo_b) * th.nown;                              // writes
  }
  moved += 5.0 * rb * nrec;
  // resident LDS positions of the touched nodes (2 B each)
  if (c->res_sstride > 0)
    for (const fed::TileHdr &th : T.tiles) moved += 2.0 * th.cum_n[1];
  I.moved_bytes_per_launch = moved;
  // resident operators that do not stay on chip (the elements that run before
  // the halo wait, or all): every tile's copies, every step
  I.reread_bytes_per_step =
      c->resident && c->op ? (double)c->hw * rb * (double)(c->Eexp - c->res_oph_elems) : 0.0;
  *out = c.release();
  return FED_OK;
}

int fed_dt(const fed_ctx *c, double *dt_crit, double *dt_used, int64_t n) {
  if (!c) return fail(FED_E_ARG, "null ctx");
  if (n < c->ninst) return fail(FED_E_ARG, "arrays hold %lld entries, need %lld", (long long)n,
                                (long long)c->ninst);
  for (int64_t i = 0; i < c->ninst; i++) {
    if (dt_crit) dt_crit[i] = c->dt_crit[i];
    if (dt_used) dt_used[i] = c->dt_used[i];
  }
  return FED_OK;
}

int fed_info_get(const fed_ctx *c, fed_info *out) {
  if (!c || !out) return fail(FED_E_ARG, "null argument");
  *out = c->info;
  out->device_bytes = (int64_t)c->pool.total;
  return FED_OK;
}

int fed_set_temperature(fed_ctx *c, const double *T, int32_t on_device, void *stream) {
  if (!c || !T) return fail(FED_E_ARG, "null argument");
  hipStream_t s = (hipStream_t)stream;
  const double *src = T;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(c->d_Tuser, T, sizeof(double) * c->N, hipMemcpyHostToDevice, s));
    src = c->d_Tuser;
  }
  c->cur = 0;
  HIPCHK(fed::launch_set_T(c->prec, c->N, src, c->d_perm, c->d_T[0], c->d_lo[0], c->ndir,
                           c->d_dir_node, c->d_dir_T, s));
  c->steps = 0;
  c->have_T = true;
  c->kept_ok = c->keep_states && c->resident && c->ckpt_every > 0;
  HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
  HIPCHK(fed::launch_health(c->d_health, 0, 0, s));
  if (c->resident) HIPCHK(hipMemsetAsync(c->d_rerr, 0, sizeof(int), s));
  if (c->ckpt_every > 0) {
    int rc = save_checkpoint(c, 0, s);
    if (rc) return rc;
  }
  if (!on_device) HIPCHK(hipStreamSynchronize(s));  // the host buffer may be reused
  return FED_OK;
}

}  // extern "C"

namespace {

// nsteps steps in launches of up to K steps, no checkpoint handling
// With check_every > 0, launches end at its multiples and the step that
// reaches one checks the energy balance; that step runs in the one-step
// kernel (whose results are bitwise those of the others), the only one that
// takes the check.
int64_t check_cut(const fed_ctx *c, int64_t done, int64_t k) {
  if (c->check_every <= 0) return k;
  return std::min<int64_t>(k, c->check_every - done % c->check_every);
}
bool energy_at(const fed_ctx *c, int64_t end) {
  return c->check_every > 0 && end % c->check_every == 0;
}

// one step in the one-step kernel from step count st, with the energy check
int energy_step(fed_ctx *c, int64_t st, hipStream_t s) {
  fed::StepArgs a = c->step_args(c->cur, 1);
  c->health_args(a, st, true);
  if (c->ps_rows > 0) a.rP = c->ps_row(st);
  HIPCHK(fed::launch_step(a, s));
  c->cur ^= 1;
  if (c->resident && c->keep_states && c->ckpt_every > 0) {
    // the step's state into the kept states, as a resident launch stores it
    const int64_t g = st / c->ckpt_every, i = st % c->ckpt_every + 1;
    int rc = seg_buffer(c, g);
    if (rc) return rc;
    const size_t hb = (size_t)c->rb * c->N;
    HIPCHK(hipMemcpyAsync((char *)c->segbuf[g] + hb * i, c->d_T[c->cur], hb,
                          hipMemcpyDeviceToDevice, s));
  }
  return FED_OK;
}

int run_steps(fed_ctx *c, int64_t nsteps, hipStream_t s) {
  if (c->resident) {
    for (int64_t n = nsteps; n > 0;) {
      const int64_t st = c->steps + nsteps - n;
      const int kc = (int)check_cut(c, st, std::min<int64_t>(n, 1 << 30));
      const bool chk = energy_at(c, st + kc);
      // the check step itself runs in the one-step kernel
      const int k = chk ? kc - 1 : kc;
      if (k > 0) {
        fed::StepArgs a = c->step_args(c->cur, 1);
        a.lds = c->res_lds;
        c->health_args(a, st, false);
        const int fin = c->cur ^ (k & 1);
        fed::ResArgs r{k, c->spin_limit, c->xtag, c->d_exported, {c->d_X[0], c->d_X[1]}, c->d_rerr,
                       c->d_T[fin], c->d_lo[fin], nullptr, 0};
        r.split = c->res_split;
        r.tag_skew = c->tag_skew;
        r.nvals = c->res_nv ? 1 : 0;
        r.ophalo = c->res_oph ? 1 : 0;
        r.sigma = c->d_sigma;
        r.sstride = c->res_sstride;
        r.ent_sigma = c->d_ent_sigma;
        if (c->keep_states && c->ckpt_every > 0) {
          // fed_step breaks launches at checkpoints: this one stays inside segment g
          const int64_t g = st / c->ckpt_every, i0 = st % c->ckpt_every;
          int rc = seg_buffer(c, g);
          if (rc) return rc;
          r.seg = (char *)c->segbuf[g] + (size_t)c->rb * c->N * i0;
          r.segN = c->N;
        }
        if (c->ps_rows > 0) {
          r.pts = c->d_psP;
          r.pts_nrec = c->nrec;
          r.pts_row = (int)(st % c->ps_rows);
          r.pts_nrows = (int)c->ps_rows;
        }
        HIPCHK(fed::launch_resident(a, r, s));
        // the launch wrote tags up to xtag + k: the next one starts beyond them
        c->xtag += (unsigned)k + 1u;
        c->cur = fin;
      }
      if (chk) {
        int rc = energy_step(c, st + k, s);
        if (rc) return rc;
      }
      n -= kc;
    }
    c->steps += nsteps;
    return FED_OK;
  }
  c->kept_ok = false;  // one-step launches keep no states
  for (int64_t n = nsteps; n > 0;) {
    // under a point-load schedule every step takes its own record powers: one
    // step per launch
    const int64_t st = c->steps + nsteps - n;
    const int kc = c->ps_rows > 0 ? 1 : (int)check_cut(c, st, std::min<int64_t>(c->K, n));
    const bool chk = energy_at(c, st + kc);
    const int k = chk ? kc - 1 : kc;
    if (k > 0) {
      fed::StepArgs a = c->step_args(c->cur, k);
      c->health_args(a, st, false);
      if (c->ps_rows > 0) a.rP = c->ps_row(st);
      HIPCHK(fed::launch_step(a, s));
      c->cur ^= 1;
    }
    if (chk) {
      int rc = energy_step(c, st + k, s);
      if (rc) return rc;
    }
    n -= kc;
  }
  c->steps += nsteps;
  return FED_OK;
}

// the kept-states buffer of checkpoint segment g, (ckpt_every + 1) hi vectors
// (allocated on first use)
int seg_buffer(fed_ctx *c, int64_t g) {
  if ((int64_t)c->segbuf.size() <= g) c->segbuf.resize(g + 1, nullptr);
  if (!c->segbuf[g])
    HIPCHK(c->pool.alloc(&c->segbuf[g], (size_t)c->rb * c->N * (c->ckpt_every + 1)));
  return FED_OK;
}

// copies the current state into checkpoint slot i (allocating it on first use)
int save_checkpoint(fed_ctx *c, int64_t i, hipStream_t s) {
  if ((int64_t)c->ck_hi.size() <= i) {
    c->ck_hi.resize(i + 1, nullptr);
    c->ck_lo.resize(i + 1, nullptr);
  }
  const size_t hb = (size_t)c->rb * c->N;
  if (!c->ck_hi[i]) HIPCHK(c->pool.alloc(&c->ck_hi[i], hb));
  HIPCHK(hipMemcpyAsync(c->ck_hi[i], c->d_T[c->cur], hb, hipMemcpyDeviceToDevice, s));
  if (c->keep_states) {
    // row 0 of the segment's kept states
    int rc = seg_buffer(c, i);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(c->segbuf[i], c->d_T[c->cur], hb, hipMemcpyDeviceToDevice, s));
  }
  if (c->prec == FED_FP32C) {
    if (!c->ck_lo[i]) HIPCHK(c->pool.alloc(&c->ck_lo[i], sizeof(float) * c->N));
    HIPCHK(hipMemcpyAsync(c->ck_lo[i], c->d_lo[c->cur], sizeof(float) * c->N,
                          hipMemcpyDeviceToDevice, s));
  }
  return FED_OK;
}

}  // namespace

extern "C" {

int fed_step(fed_ctx *c, int64_t nsteps, void *stream) {
  if (!c) return fail(FED_E_ARG, "null ctx");
  if (!c->have_T) return fail(FED_E_STATE, "fed_set_temperature must come first");
  if (nsteps < 0) return fail(FED_E_ARG, "nsteps < 0");
  hipStream_t s = (hipStream_t)stream;
  if (c->ckpt_every <= 0) return run_steps(c, nsteps, s);
  // break the launches at checkpoint steps and save the state there
  while (nsteps > 0) {
    int64_t chunk = std::min(nsteps, c->ckpt_every - c->steps % c->ckpt_every);
    int rc = run_steps(c, chunk, s);
    if (rc) return rc;
    nsteps -= chunk;
    if (c->steps % c->ckpt_every == 0) {
      rc = save_checkpoint(c, c->steps / c->ckpt_every, s);
      if (rc) return rc;
    }
  }
  return FED_OK;
}

int fed_step_graph(fed_ctx *c, int64_t nsteps, int32_t graph_steps, void *stream) {
  if (!c) return fail(FED_E_ARG, "null ctx");
  if (!c->have_T) return fail(FED_E_STATE, "fed_set_temperature must come first");
  if (nsteps < 0 || graph_steps < 0) return fail(FED_E_ARG, "negative count");
  // checkpoints break launches; a resident launch already runs all the steps; a
  // point-load schedule gives every step its own launch arguments; energy checks
  // with K-step launches split launches (replays check at their last step only
  // with one-step launches)
  if (c->ckpt_every > 0 || c->resident || c->ps_rows > 0 || (c->check_every > 0 && c->K > 1))
    return fed_step(c, nsteps, stream);
  hipStream_t s = (hipStream_t)stream;
  // an even number of K-step launches, so every replay starts on the same buffer
  int64_t want = graph_steps ? graph_steps : 100;
  int launches = (int)std::max<int64_t>(2, (want + c->K - 1) / c->K);
  launches += launches & 1;
  int gs = launches * c->K;
  if (nsteps < gs) return fed_step(c, nsteps, stream);
  if (c->gexec && (c->gsteps != gs || c->gparity != c->cur)) c->drop_graph();
  if (!c->gexec) {
    // capture on a private stream (the caller's may be the legacy null stream,
    // which cannot be captured); the graph is then launched on the caller's stream
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = c->cap_stream;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int par = c->cur;
    for (int i = 0; i <= launches; i++) {
      hipError_t e;
      if (i < launches) {
        // health: steps counted from the replay's base; the replay's last
        // launch checks the energy balance
        fed::StepArgs a = c->step_args(par, c->K);
        c->health_args(a, (long long)i * c->K, c->check_every > 0 && i == launches - 1);
        a.hbase = 1;
        e = fed::launch_step(a, cs);
      } else {
        e = fed::launch_health(c->d_health, 2, gs, cs);  // the next replay's base
      }
      if (e != hipSuccess) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cs, &g);
        if (g) (void)hipGraphDestroy(g);
        return fail(FED_E_HIP, "capture launch failed: %s", hipGetErrorString(e));
      }
      par ^= 1;
    }
    HIPCHK(hipStreamEndCapture(cs, &c->graph));
    HIPCHK(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    c->gsteps = gs;
    c->gparity = c->cur;
  }
  int64_t reps = nsteps / gs;
  HIPCHK(fed::launch_health(c->d_health, 1, c->steps, s));
  for (int64_t r = 0; r < reps; r++) HIPCHK(hipGraphLaunch(c->gexec, s));
  c->steps += reps * gs;
  return run_steps(c, nsteps - reps * gs, s);
}

int fed_get_temperature(fed_ctx *c, double *T, int32_t on_device, void *stream) {
  if (!c || !T) return fail(FED_E_ARG, "null argument");
  if (!c->have_T) return fail(FED_E_STATE, "no temperature set");
  hipStream_t s = (hipStream_t)stream;
  const double wlo = c->win_lo, whi = c->win_hi;
  // the readout check covers the current state only
  HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
  HIPCHK(fed::launch_check(c->prec, c->N, c->d_T[c->cur], c->d_lo[c->cur], wlo, whi, c->d_flag, s));
  double *dst = on_device ? T : c->d_Tuser;
  HIPCHK(fed::launch_get_T(c->prec, c->N, c->d_perm, c->d_T[c->cur], c->d_lo[c->cur], dst, s));
  int flag = 0;
  if (!on_device)
    HIPCHK(hipMemcpyAsync(T, c->d_Tuser, sizeof(double) * c->N, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  fed::Health h{};
  HIPCHK(hipMemcpyAsync(&h, c->d_health, sizeof(h), hipMemcpyDeviceToHost, s));
  int rerr = 0;
  if (c->resident) HIPCHK(hipMemcpyAsync(&rerr, c->d_rerr, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (rerr)
    return fail(FED_E_HIP, "resident stepping: a tile gave up waiting for a neighbouring tile; "
                           "the temperatures are invalid");
  if (h.first_bad != ~0ull)
    return fail(FED_E_UNSTABLE,
                "health check: a temperature left [%g, %g] or was not finite after step %llu "
                "(the stability bound holds for [T_lo, T_hi]; %lld steps taken)",
                wlo, whi, h.first_bad, (long long)c->steps);
  if (flag)
    return fail(FED_E_UNSTABLE,
                "health check: a temperature is non-finite or outside [%g, %g] after %lld steps",
                wlo, whi, (long long)c->steps);
  if (c->energy_tol > 0 && !(h.energy_max <= c->energy_tol))
    return fail(FED_E_UNSTABLE,
                "health check: energy residual %.3g at step %lld exceeds energy_tol %.3g",
                h.energy_max, h.energy_step, c->energy_tol);
  return FED_OK;
}

int fed_health_get(fed_ctx *c, fed_health *out, void *stream) {
  if (!c || !out) return fail(FED_E_ARG, "null argument");
  hipStream_t s = (hipStream_t)stream;
  fed::Health h{};
  HIPCHK(hipMemcpyAsync(&h, c->d_health, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  out->steps = c->steps;
  out->first_bad_step = h.first_bad == ~0ull ? -1 : (int64_t)h.first_bad;
  out->window_lo = c->win_lo;
  out->window_hi = c->win_hi;
  out->energy_residual = h.energy_max;
  out->energy_step = h.energy_step;
  out->energy_checks = h.checks;
  return FED_OK;
}

int fed_steps_taken(const fed_ctx *c, int64_t *steps) {
  if (!c || !steps) return fail(FED_E_ARG, "null argument");
  *steps = c->steps;
  return FED_OK;
}

int fed_get_state(fed_ctx *c, void *hi, void *lo, int64_t *step, void *stream) {
  if (!c || !hi) return fail(FED_E_ARG, "null argument");
  if (!c->have_T) return fail(FED_E_STATE, "no temperature set");
  hipStream_t s = (hipStream_t)stream;
  const int rb = c->rb;
  // staged in caller order through the FP64 readout buffer (8 bytes a node)
  void *tmp = c->d_Tuser;
  HIPCHK(fed::launch_permute(rb, c->N, c->d_perm, c->d_T[c->cur], tmp, 0, s));
  HIPCHK(hipMemcpyAsync(hi, tmp, (size_t)rb * c->N, hipMemcpyDeviceToHost, s));
  if (lo && c->prec == FED_FP32C) {
    HIPCHK(fed::launch_permute(4, c->N, c->d_perm, c->d_lo[c->cur], tmp, 0, s));
    HIPCHK(hipMemcpyAsync(lo, tmp, sizeof(float) * c->N, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  if (step) *step = c->steps;
  return FED_OK;
}

int fed_set_state(fed_ctx *c, const void *hi, const void *lo, int64_t step, void *stream) {
  if (!c || !hi) return fail(FED_E_ARG, "null argument");
  if (c->prec == FED_FP32C && !lo) return fail(FED_E_ARG, "FP32C state needs lo");
  hipStream_t s = (hipStream_t)stream;
  const int rb = c->rb;
  void *tmp = c->d_Tuser;  // caller-order staging, as in fed_get_state
  c->cur = 0;
  HIPCHK(hipMemcpyAsync(tmp, hi, (size_t)rb * c->N, hipMemcpyHostToDevice, s));
  HIPCHK(fed::launch_permute(rb, c->N, c->d_perm, tmp, c->d_T[0], 1, s));
  if (c->prec == FED_FP32C) {
    HIPCHK(hipMemcpyAsync(tmp, lo, sizeof(float) * c->N, hipMemcpyHostToDevice, s));
    HIPCHK(fed::launch_permute(4, c->N, c->d_perm, tmp, c->d_lo[0], 1, s));
  }
  HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
  HIPCHK(fed::launch_health(c->d_health, 0, 0, s));
  if (c->resident) HIPCHK(hipMemsetAsync(c->d_rerr, 0, sizeof(int), s));
  HIPCHK(hipStreamSynchronize(s));
  c->steps = step;
  c->kept_ok = false;
  c->have_T = true;
  return FED_OK;
}

int fed_checkpoint_every(fed_ctx *c, int64_t every) {
  if (!c) return fail(FED_E_ARG, "null ctx");
  if (every < 0) return fail(FED_E_ARG, "every < 0");
  if (every != c->ckpt_every || every == 0) {
    // the buffers are reused (and overwritten) while the interval stays the same
    for (void *p : c->ck_hi) c->pool.release(p);
    for (void *p : c->ck_lo) c->pool.release(p);
    c->ck_hi.clear();
    c->ck_lo.clear();
    for (void *p : c->segbuf) c->pool.release(p);
    c->segbuf.clear();
  }
  c->ckpt_every = every;
  c->have_T = false;  // the checkpoint of step 0 is taken by fed_set_temperature
  return FED_OK;
}

int fed_set_params(fed_ctx *c, const double *kscale, const double *elem_c, const double *face_h,
                   int32_t on_device, void *stream) {
  if (!c) return fail(FED_E_ARG, "null ctx");
  hipStream_t s = (hipStream_t)stream;
  const int64_t E = c->E, N = c->N, nf = c->nf;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  // validate on the host
  std::vector<double> ks, ec, fh;
  if (kscale) {
    ks.resize(E);
    HIPCHK(hipMemcpy(ks.data(), kscale, sizeof(double) * E, kind));
    for (int64_t e = 0; e < E; e++)
      if (!(ks[e] > 0) || !std::isfinite(ks[e])) return fail(FED_E_ARG, "kscale[%lld] invalid", (long long)e);
  }
  if (elem_c) {
    if (c->tdc) return fail(FED_E_ARG, "per-element heat capacity needs c1 = 0");
    ec.resize(E);
    HIPCHK(hipMemcpy(ec.data(), elem_c, sizeof(double) * E, kind));
    for (int64_t e = 0; e < E; e++)
      if (!(ec[e] > 0) || !std::isfinite(ec[e])) return fail(FED_E_ARG, "elem_c[%lld] invalid", (long long)e);
  }
  if (face_h) {
    if (nf == 0) return fail(FED_E_ARG, "the problem has no faces");
    fh.resize(nf);
    HIPCHK(hipMemcpy(fh.data(), face_h, sizeof(double) * nf, kind));
    for (int64_t f = 0; f < nf; f++)
      if (!(fh[f] >= 0) || !std::isfinite(fh[f])) return fail(FED_E_ARG, "face_h[%lld] invalid", (long long)f);
  }
  // re-derive on the GPU
  if (kscale) HIPCHK(hipMemcpyAsync(c->d_kscale, ks.data(), sizeof(double) * E, hipMemcpyHostToDevice, s));
  if (elem_c) {
    if (!c->d_ec0) HIPCHK(c->pool.alloc((void **)&c->d_ec0, sizeof(double) * E));
    HIPCHK(hipMemcpyAsync(c->d_ec0, ec.data(), sizeof(double) * E, hipMemcpyHostToDevice, s));
  }
  if (face_h) HIPCHK(hipMemcpyAsync(c->d_fh, fh.data(), sizeof(double) * nf, hipMemcpyHostToDevice, s));
  fed::MassArgs ma{N, c->ne, c->d_incp, c->d_ince, c->d_mats, c->d_emat, c->d_ec0, c->d_V,
                   c->T_lo, c->T_hi, c->d_M0, c->d_M1, c->d_Cmin, c->fc_min};
  HIPCHK(fed::launch_mass(ma, s));
  if (c->nrec > 0) {
    fed::BndArgs ba{0, c->nfn, c->d_faces, nullptr, nullptr, nullptr, c->d_fh, c->d_fTa,
                    c->d_feps, c->d_fq, c->d_farea, c->nrec, c->d_recptr, c->d_recitem,
                    c->d_ptW, c->d_b64[0], c->d_b64[1], c->d_b64[2], c->d_b64[3], nullptr};
    HIPCHK(fed::launch_bnd(ba, s));  // nf = 0: face areas are kept, records recomputed
  }
  HIPCHK(hipMemsetAsync(c->d_lam, 0, sizeof(unsigned long long) * 2 * c->ninst, s));
  fed::DtArgs da{c->ne, E, c->nrec, c->d_lamgeo, c->d_kscale, c->d_mats, c->d_emat, c->d_ec0,
                 c->d_einst, c->d_recnode, c->d_ninst, c->d_b64[0], c->d_b64[2], c->d_Cmin,
                 c->T_lo, c->T_hi, c->Tz, c->d_lam, c->d_lam + c->ninst, c->fk_max, c->fc_min};
  HIPCHK(fed::launch_dt(da, s));
  std::vector<unsigned long long> lam(2 * c->ninst);
  HIPCHK(hipMemcpyAsync(lam.data(), c->d_lam, lam.size() * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int64_t i = 0; i < c->ninst; i++) {
    double le, lb;
    std::memcpy(&le, &lam[i], 8);
    std::memcpy(&lb, &lam[c->ninst + i], 8);
    c->dt_crit[i] = le + lb > 0 ? 2.0 / (le + lb) : INFINITY;
    if (c->dt_used[i] > c->dt_crit[i] && !c->allow_unstable)
      return fail(FED_E_UNSTABLE, "dt %.6g exceeds the new dt_crit %.6g (instance %lld)",
                  c->dt_used[i], c->dt_crit[i], (long long)i);
  }
  int rc = derive_window(c, s);  // the bound moved: so does the window it allows
  if (rc) return rc;
  fed::NodeArrArgs na{c->prec, N, c->nrec, c->d_M0, c->d_M1, c->d_dtinst, c->d_ninst, c->d_isdir,
                      c->d_b64[0], c->d_b64[1], c->d_b64[2], c->d_b64[4], c->d_b64[3],
                      c->d_alpha, c->d_beta, c->d_rA, c->d_rAT, c->d_reA, c->d_rTa, c->d_rP};
  HIPCHK(fed::launch_node_arrays(na, s));
  HIPCHK(fed::launch_expand_H(c->prec == FED_FP64 ? 1 : 0, c->hw, c->hs_from(), c->hs_to(), c->Eexp, E,
                              c->d_eorig, c->d_H0,
                              c->d_kscale, c->d_H, s));
  HIPCHK(hipStreamSynchronize(s));
  return FED_OK;
}

int fed_set_bc(fed_ctx *c, const double *face_Ta, const double *face_q, const double *pt_W,
               int32_t on_device, void *stream) {
  if (!c) return fail(FED_E_ARG, "null ctx");
  if ((face_Ta || face_q) && c->nf == 0) return fail(FED_E_ARG, "the problem has no faces");
  if (pt_W && c->npt == 0) return fail(FED_E_ARG, "the problem has no point loads");
  if (pt_W && c->ps_rows > 0)
    return fail(FED_E_STATE, "a point-load schedule is set (fed_set_point_schedule)");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nf = c->nf;
  if (!on_device) {
    for (int64_t f = 0; f < nf; f++) {
      if (face_Ta && !std::isfinite(face_Ta[f])) return fail(FED_E_ARG, "face_Ta[%lld] invalid", (long long)f);
      if (face_q && !std::isfinite(face_q[f])) return fail(FED_E_ARG, "face_q[%lld] invalid", (long long)f);
    }
    for (int64_t i = 0; pt_W && i < c->npt; i++)
      if (!std::isfinite(pt_W[i])) return fail(FED_E_ARG, "pt_W[%lld] invalid", (long long)i);
    if (face_Ta && c->has_rad) {
      // radiating faces that share a node must share Ta (one radiation ambient per node)
      std::vector<double> ta(c->N, 0.0);
      std::vector<uint8_t> set(c->N, 0);
      for (int64_t f = 0; f < nf; f++) {
        if (!(c->h_feps[f] > 0)) continue;
        for (int b = 0; b < c->nfn; b++) {
          const int32_t k = c->h_faces[f * c->nfn + b];
          if (set[k] && ta[k] != face_Ta[f])
            return fail(FED_E_ARG, "radiating faces at node %d have different Ta", k);
          set[k] = 1;
          ta[k] = face_Ta[f];
        }
      }
    }
  }
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (face_Ta) HIPCHK(hipMemcpyAsync(c->d_fTa, face_Ta, sizeof(double) * nf, kind, s));
  if (face_q) HIPCHK(hipMemcpyAsync(c->d_fq, face_q, sizeof(double) * nf, kind, s));
  if (pt_W) HIPCHK(hipMemcpyAsync(c->d_ptW, pt_W, sizeof(double) * c->npt, kind, s));
  if (c->nrec > 0 && (face_Ta || face_q || pt_W)) {
    fed::BndArgs ba{0, c->nfn, c->d_faces, nullptr, nullptr, nullptr, c->d_fh, c->d_fTa,
                    c->d_feps, c->d_fq, c->d_farea, c->nrec, c->d_recptr, c->d_recitem,
                    c->d_ptW, c->d_b64[0], c->d_b64[1], c->d_b64[2], c->d_b64[3], c->d_b64[4]};
    HIPCHK(fed::launch_bnd(ba, s));
    // the boundary records only (N = 0): alpha and beta do not depend on the loads
    fed::NodeArrArgs na{c->prec, 0, c->nrec, c->d_M0, c->d_M1, c->d_dtinst, c->d_ninst,
                        c->d_isdir, c->d_b64[0], c->d_b64[1], c->d_b64[2], c->d_b64[4],
                        c->d_b64[3], c->d_alpha, c->d_beta, c->d_rA, c->d_rAT, c->d_reA,
                        c->d_rTa, c->d_rP};
    HIPCHK(fed::launch_node_arrays(na, s));
    // the schedule's rows hold the face fluxes too
    if (face_q && c->ps_rows > 0)
      HIPCHK(fed::launch_point_rows(c->prec == FED_FP64 ? 1 : 0, ba, c->ps_rows, c->npt,
                                    c->d_psW, c->d_psP, s));
  }
  if (!on_device) HIPCHK(hipStreamSynchronize(s));  // the host arrays may be reused
  return FED_OK;
}

int fed_set_point_schedule(fed_ctx *c, const double *W, int64_t n_rows, int32_t on_device,
                           void *stream) {
  if (!c) return fail(FED_E_ARG, "null ctx");
  if (n_rows < 0 || n_rows > INT32_MAX) return fail(FED_E_ARG, "n_rows %lld out of range", (long long)n_rows);
  if (n_rows > 0 && !W) return fail(FED_E_ARG, "null W");
  if (n_rows > 0 && c->npt == 0) return fail(FED_E_ARG, "the problem has no point loads");
  hipStream_t s = (hipStream_t)stream;
  if (n_rows > 0 && !on_device)
    for (int64_t i = 0; i < n_rows * c->npt; i++)
      if (!std::isfinite(W[i])) return fail(FED_E_ARG, "W[%lld] invalid", (long long)i);
  if (c->ps_rows != n_rows) {
    // launches already queued may still read the old tables
    HIPCHK(hipDeviceSynchronize());
    c->pool.release(c->d_psW);
    c->pool.release(c->d_psP);
    c->d_psW = nullptr;
    c->d_psP = nullptr;
    c->ps_rows = 0;
    if (n_rows == 0) return FED_OK;
    HIPCHK(c->pool.alloc((void **)&c->d_psW, sizeof(double) * n_rows * c->npt));
    HIPCHK(c->pool.alloc(&c->d_psP, (size_t)c->rb * n_rows * c->nrec));
  } else if (n_rows == 0) {
    return FED_OK;
  }
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIPCHK(hipMemcpyAsync(c->d_psW, W, sizeof(double) * n_rows * c->npt, kind, s));
  fed::BndArgs ba{0, c->nfn, c->d_faces, nullptr, nullptr, nullptr, c->d_fh, c->d_fTa,
                  c->d_feps, c->d_fq, c->d_farea, c->nrec, c->d_recptr, c->d_recitem,
                  c->d_ptW, c->d_b64[0], c->d_b64[1], c->d_b64[2], c->d_b64[3], c->d_b64[4]};
  HIPCHK(fed::launch_point_rows(c->prec == FED_FP64 ? 1 : 0, ba, n_rows, c->npt, c->d_psW,
                                c->d_psP, s));
  c->ps_rows = n_rows;
  if (!on_device) HIPCHK(hipStreamSynchronize(s));  // the host array may be reused
  return FED_OK;
}

int fed_keep_states(fed_ctx *c, int32_t on) {
  if (!c) return fail(FED_E_ARG, "null ctx");
  if (on && !c->resident) return fail(FED_E_STATE, "kept states need a resident context");
  if (on && c->ckpt_every <= 0) return fail(FED_E_STATE, "checkpointing is off (fed_checkpoint_every)");
  c->keep_states = on != 0;
  if (!c->keep_states) {
    for (void *p : c->segbuf) c->pool.release(p);
    c->segbuf.clear();
  }
  c->have_T = false;  // the states are kept from fed_set_temperature on
  c->kept_ok = false;
  return FED_OK;
}

int fed_test_waits(fed_ctx *c, int32_t spin_limit, int32_t never_match) {
  if (!c) return fail(FED_E_ARG, "null ctx");
  if (spin_limit < 0) return fail(FED_E_ARG, "spin_limit < 0");
  if (!c->resident) return fail(FED_E_STATE, "not a resident context");
  c->spin_limit = spin_limit ? spin_limit : 1 << 22;
  c->tag_skew = never_match ? 0x40000000u : 0u;
  return FED_OK;
}

int fed_temperature_range(fed_ctx *c, double *tmin, double *tmax, void *stream) {
  if (!c || !tmin || !tmax) return fail(FED_E_ARG, "null argument");
  if (!c->have_T) return fail(FED_E_STATE, "no temperature set");
  hipStream_t s = (hipStream_t)stream;
  unsigned long long init[2] = {~0ull, 0ull}, keys[2];
  int nan = 0;
  HIPCHK(hipMemcpyAsync(c->d_rkeys, init, sizeof(init), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(c->d_rnan, 0, sizeof(int), s));
  HIPCHK(fed::launch_range(c->prec, c->N, c->d_T[c->cur], c->d_lo[c->cur], c->d_rkeys, c->d_rnan, s));
  HIPCHK(hipMemcpyAsync(keys, c->d_rkeys, sizeof(keys), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&nan, c->d_rnan, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  auto value = [](unsigned long long k) {
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    double v;
    std::memcpy(&v, &b, 8);
    return v;
  };
  *tmin = nan ? NAN : value(keys[0]);
  *tmax = nan ? NAN : value(keys[1]);
  return FED_OK;
}

int fed_set_range(fed_ctx *c, double T_lo, double T_hi, void *stream) {
  if (!c) return fail(FED_E_ARG, "null ctx");
  if (!std::isfinite(T_lo) || !std::isfinite(T_hi) || !(T_hi > T_lo))
    return fail(FED_E_ARG, "need finite T_lo < T_hi");
  for (size_t i = 0; i < c->h_mats.size(); i++) {
    const fed_material &q = c->h_mats[i];
    if (!(q.c0 + q.c1 * T_lo > 0 && q.c0 + q.c1 * T_hi > 0) ||
        !(q.s0 + q.s1 * T_lo > 0 && q.s0 + q.s1 * T_hi > 0))
      return fail(FED_E_ARG, "material %d: c(T) or D(T) not positive on [%g, %g]", (int)i, T_lo, T_hi);
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<double> dtc;
  int rc = bound_dt(c, T_lo, T_hi, dtc, s);
  if (rc) return rc;
  c->dt_crit = dtc;
  c->T_lo = T_lo;
  c->T_hi = T_hi;
  c->fk_max = c->nkt ? table_extreme(c->h_ktab_T, c->h_ktab_f, T_lo, T_hi, true) : 1.0;
  c->fc_min = c->nct ? table_extreme(c->h_ctab_T, c->h_ctab_f, T_lo, T_hi, false) : 1.0;
  rc = derive_window(c, s);
  if (rc) return rc;
  // the new window starts clean
  HIPCHK(fed::launch_health(c->d_health, 3, 0, s));
  HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
  HIPCHK(hipStreamSynchronize(s));
  for (int64_t i = 0; i < c->ninst; i++)
    if (c->dt_used[i] > c->dt_crit[i] && !c->allow_unstable)
      return fail(FED_E_UNSTABLE, "dt %.6g exceeds dt_crit %.6g on [%g, %g] (instance %lld)",
                  c->dt_used[i], c->dt_crit[i], T_lo, T_hi, (long long)i);
  return FED_OK;
}

}  // extern "C"

namespace {

// Places the adjoint's work arrays through place(void **slot, size_t bytes), in
// a fixed order; the segment's states only when some segment is recomputed.
template <typename F>
int adj_work_layout(const fed_ctx *c, bool need_seg, fed::AdjWork &w, F place) {
  const int64_t N = c->N, E = c->E;
  const size_t rb = (size_t)c->rb;
  const bool c32 = c->prec == FED_FP32C;
  if (need_seg) {
    HIPCHK(place(&w.seg, rb * N * (c->ckpt_every + 1)));
    if (c32)
      for (int i = 0; i < 2; i++) HIPCHK(place((void **)&w.seglo[i], sizeof(float) * N));
  }
  for (int i = 0; i < 2; i++) {
    HIPCHK(place(&w.lamb[i], rb * N));
    if (c32) HIPCHK(place((void **)&w.lamlo[i], sizeof(float) * N));
  }
  HIPCHK(place((void **)&w.S0, sizeof(double) * std::max<int64_t>(c->nrec, 1)));
  HIPCHK(place((void **)&w.S1, sizeof(double) * std::max<int64_t>(c->nrec, 1)));
  HIPCHK(place((void **)&w.gk, sizeof(double) * E));
  HIPCHK(place((void **)&w.gc, sizeof(double) * E));
  HIPCHK(place((void **)&w.gh, sizeof(double) * std::max<int64_t>(c->nf, 1)));
  HIPCHK(place(&w.rdt, rb * N));
  HIPCHK(place(&w.mV, rb * E));
  return FED_OK;
}

int backward_checks(const fed_ctx *c, const double *dL_dT) {
  if (!c || !dL_dT) return fail(FED_E_ARG, "null argument");
  if (!c->have_T) return fail(FED_E_STATE, "no forward run");
  if (c->ckpt_every <= 0) return fail(FED_E_STATE, "checkpointing is off (fed_checkpoint_every)");
  if (c->adj_lds > c->max_lds)
    return fail(FED_E_MESH, "adjoint tiles need %d bytes of LDS; use smaller tile_nodes", c->adj_lds);
  return FED_OK;
}

// The adjoint of the steps taken, with the work arrays w (fed_backward: the
// context's; fed_backward_noalloc: the static scratch).
int backward_run(fed_ctx *c, const fed::AdjWork &w, const double *dL_dT, double *g_logk,
                 double *g_c, double *g_h, double *dL_dT0, int32_t on_device, hipStream_t s) {
  const int64_t N = c->N, E = c->E, ck = c->ckpt_every, steps = c->steps;
  const int rb = c->rb;
  HIPCHK(fed::launch_adjoint_coefs(c->prec == FED_FP64 ? 1 : 0, N, E, c->ne, c->d_dtinst,
                                   c->d_ninst, c->d_mats, c->d_emat, c->d_V, w.rdt, w.mV, s));
  HIPCHK(hipMemsetAsync(w.S0, 0, sizeof(double) * std::max<int64_t>(c->nrec, 1), s));
  HIPCHK(hipMemsetAsync(w.S1, 0, sizeof(double) * std::max<int64_t>(c->nrec, 1), s));
  HIPCHK(hipMemsetAsync(w.gk, 0, sizeof(double) * E, s));
  HIPCHK(hipMemsetAsync(w.gc, 0, sizeof(double) * E, s));
  // lambda^N = dL/dT^N in internal order
  const double *src = dL_dT;
  if (!on_device) {
    HIPCHK(hipMemcpyAsync(c->d_Tuser, dL_dT, sizeof(double) * N, hipMemcpyHostToDevice, s));
    src = c->d_Tuser;
  }
  HIPCHK(fed::launch_set_T(c->prec, N, src, c->d_perm, w.lamb[0], w.lamlo[0], 0, nullptr,
                           nullptr, s));
  int lc = 0;
  void *segb = w.seg;  // the states of the segment at hand: kept or recomputed
  auto seg = [&](int64_t i) {
    return (void *)((char *)segb + (size_t)rb * N * i);
  };
  const int64_t nseg = (steps + ck - 1) / ck;
  for (int64_t g = nseg - 1; g >= 0; g--) {
    const int64_t n0 = g * ck, n1 = std::min(steps, n0 + ck);
    if (g >= (int64_t)c->ck_hi.size() || !c->ck_hi[g])
      return fail(FED_E_STATE, "checkpoint %lld missing", (long long)g);
    // the segment's states T^{n0..n1}: kept by the forward launches, or
    // recomputed from its checkpoint
    const bool kept = c->kept_ok && g < (int64_t)c->segbuf.size() && c->segbuf[g];
    segb = kept ? c->segbuf[g] : w.seg;
    if (!kept) {
      HIPCHK(hipMemcpyAsync(seg(0), c->ck_hi[g], (size_t)rb * N, hipMemcpyDeviceToDevice, s));
      if (c->prec == FED_FP32C)
        HIPCHK(hipMemcpyAsync(w.seglo[0], c->ck_lo[g], sizeof(float) * N,
                              hipMemcpyDeviceToDevice, s));
    }
    if (kept) {
      // nothing to recompute
    } else if (c->resident && n1 > n0) {
      // one resident launch recomputes the segment, storing every step's hi
      const int k = (int)(n1 - n0);
      fed::StepArgs a = c->step_args(0, 1);
      a.lds = c->res_lds;
      a.Tin = seg(0);
      a.loin = w.seglo[0];
      a.Tout = seg(1);  // not used by the resident kernel
      fed::ResArgs r{k, 1 << 22, c->xtag, c->d_exported, {c->d_X[0], c->d_X[1]}, c->d_rerr,
                     seg(k), w.seglo[k & 1], segb, N};
      r.split = c->res_split;
      r.nvals = c->res_nv ? 1 : 0;
      r.ophalo = c->res_oph ? 1 : 0;
      r.sigma = c->d_sigma;
      r.sstride = c->res_sstride;
      r.ent_sigma = c->d_ent_sigma;
      if (c->ps_rows > 0) {
        r.pts = c->d_psP;
        r.pts_nrec = c->nrec;
        r.pts_row = (int)(n0 % c->ps_rows);
        r.pts_nrows = (int)c->ps_rows;
      }
      HIPCHK(fed::launch_resident(a, r, s));
      c->xtag += (unsigned)k + 1u;
    } else {
      for (int64_t i = 0; i < n1 - n0; i++) {
        fed::StepArgs a = c->step_args(0, 1);
        a.Tin = seg(i);
        a.Tout = seg(i + 1);
        a.loin = w.seglo[i & 1];
        a.loout = w.seglo[(i + 1) & 1];
        if (c->ps_rows > 0) a.rP = c->ps_row(n0 + i);
        HIPCHK(fed::launch_step(a, s));
      }
    }
    // adjoint steps n1-1 .. n0
    fed::AdjArgs a{};
    a.prec = c->prec;
    a.ne = c->ne;
    a.nt = c->til.nt;
    a.nper = c->nper;
    a.block = c->block;
    a.lds = c->adj_lds;
    a.pb = c->til.pb;
    a.maxinc = c->til.maxinc;
    a.Eexp = c->Eexp;
    a.tiles = c->d_tiles;
    a.ent = c->d_ent;
    a.halo = c->d_halo;
    a.eorig = c->d_eorig;
    a.eowner = c->d_eowner;
    a.H = c->d_H;
    a.alpha = c->d_alpha;
    a.rdt = w.rdt;
    a.mV = w.mV;
    a.rA = c->d_rA;
    a.g_logk = w.gk;
    a.g_c = w.gc;
    a.S0 = w.S0;
    a.S1 = w.S1;
    a.s0 = c->s0;
    a.tdk = c->tdk;
    a.tdc = c->tdc;
    a.s1 = c->s1;
    a.Tz = c->Tz;
    a.beta = c->d_beta;
    a.reA = c->d_reA;
    a.esk = c->d_esk;
    a.ktab = c->d_ktab;
    a.ctab = c->d_ctab;
    a.nkt = c->nkt;
    a.nct = c->nct;
    a.op = c->op;
    if (c->adjres && n1 > n0) {
      // one resident launch for the segment
      const int k = (int)(n1 - n0);
      a.lds = c->adjres_lds;
      a.lamin = w.lamb[lc];
      a.lamloin = w.lamlo[lc];
      a.lamout = w.lamb[1 - lc];
      a.lamloout = w.lamlo[1 - lc];
      fed::AdjResArgs r{k, 1 << 22, c->xtag, c->d_exported, {c->d_X[0], c->d_X[1]}, c->d_rerr,
                        segb, N};
      HIPCHK(fed::launch_adjres(a, r, s));
      c->xtag += (unsigned)k + 1u;
      lc ^= 1;
      continue;
    }
    for (int64_t n = n1 - 1; n >= n0; n--) {
      a.lamin = w.lamb[lc];
      a.lamloin = w.lamlo[lc];
      a.lamout = w.lamb[1 - lc];
      a.lamloout = w.lamlo[1 - lc];
      a.Tn = seg(n - n0);
      a.Tn1 = seg(n - n0 + 1);
      HIPCHK(fed::launch_adjoint(a, s));
      lc ^= 1;
    }
  }
  if (c->nf > 0)
    HIPCHK(fed::launch_face_grad(c->nf, c->nfn, c->d_faces, c->d_perm, c->d_rec_of, c->d_farea,
                                 c->d_fTa, w.S0, w.S1, w.gh, s));
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (g_logk) HIPCHK(hipMemcpyAsync(g_logk, w.gk, sizeof(double) * E, kind, s));
  if (g_c) HIPCHK(hipMemcpyAsync(g_c, w.gc, sizeof(double) * E, kind, s));
  if (g_h && c->nf > 0) HIPCHK(hipMemcpyAsync(g_h, w.gh, sizeof(double) * c->nf, kind, s));
  if (dL_dT0) {
    double *dst = on_device ? dL_dT0 : c->d_Tuser;
    HIPCHK(fed::launch_get_T(c->prec, N, c->d_perm, w.lamb[lc], w.lamlo[lc], dst, s));
    if (!on_device)
      HIPCHK(hipMemcpyAsync(dL_dT0, c->d_Tuser, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  }
  int rerr = 0;
  if (c->resident) HIPCHK(hipMemcpyAsync(&rerr, c->d_rerr, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (rerr)
    return fail(FED_E_HIP, "resident stepping: a tile gave up waiting for a neighbouring tile; "
                           "the derivatives are invalid");
  return FED_OK;

}

// true when every segment of the run has its states kept (no recompute)
bool all_segments_kept(const fed_ctx *c) {
  if (!c->kept_ok) return false;
  const int64_t nseg = (c->steps + c->ckpt_every - 1) / c->ckpt_every;
  if ((int64_t)c->segbuf.size() < nseg) return false;
  for (int64_t g = 0; g < nseg; g++)
    if (!c->segbuf[g]) return false;
  return true;
}

}  // namespace

extern "C" {

int fed_backward(fed_ctx *c, const double *dL_dT, double *g_logk, double *g_c, double *g_h,
                 double *dL_dT0, int32_t on_device, void *stream) {
  int rc = backward_checks(c, dL_dT);
  if (rc) return rc;
  if (!c->adjw.lamb[0]) {
    // the context's work arrays, allocated on first use
    DevPool &P = c->pool;
    rc = adj_work_layout(c, true, c->adjw,
                         [&](void **slot, size_t bytes) { return P.alloc(slot, bytes); });
    if (rc) return rc;
  }
  return backward_run(c, c->adjw, dL_dT, g_logk, g_c, g_h, dL_dT0, on_device,
                      (hipStream_t)stream);
}

int fed_backward_noalloc(fed_ctx *c, const double *dL_dT, double *g_logk, double *g_c,
                         double *g_h, double *dL_dT0, int32_t on_device, void *stream) {
  int rc = backward_checks(c, dL_dT);
  if (rc) return rc;
  void *base = nullptr;
  HIPCHK(fed::scratch_address(&base));
  // the work arrays, 256-byte aligned, one after another in the scratch
  size_t used = 0;
  fed::AdjWork w;
  auto carve = [&](void **slot, size_t bytes) {
    used = (used + 255) & ~(size_t)255;
    *slot = used + bytes <= fed::kScratchBytes ? (char *)base + used : nullptr;
    used += bytes;
    return hipSuccess;
  };
  rc = adj_work_layout(c, !all_segments_kept(c), w, carve);
  if (rc) return rc;
  if (used > fed::kScratchBytes)
    return fail(FED_E_ARG,
                "fed_backward_noalloc: the adjoint's work arrays need %zu bytes, the scratch "
                "holds %zu; use fed_backward, a shorter checkpoint interval or kept states",
                used, fed::kScratchBytes);
  return backward_run(c, w, dL_dT, g_logk, g_c, g_h, dL_dT0, on_device, (hipStream_t)stream);
}

void fed_destroy(fed_ctx *c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  delete c;
}

}  // extern "C"
