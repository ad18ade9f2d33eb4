// Launchers of the FED-FEM HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fedfem.h"
#include "fed_internal.h"

namespace fed {

// Material record, same layout as the public fed_material.
struct MatDev {
  double rho, c0, c1;
  double k[6];
  double s0, s1;
};

struct GeomArgs {
  int ne;
  int64_t E;
  const double *x, *y, *z;
  const int32_t *conn;     // caller ids, [ne * E]
  const MatDev *mats;
  const int32_t *emat;     // nullable
  const double *ek;        // nullable, [6 * E]
  double *H0;              // [W * E] element operator without per-element factor: W = 6
                           // (folded 3x3), 27 (uniform-gradient hexahedron: 21 mean
                           // gradient values, then V D) or 40 (then also kappa and the
                           // 12 values h_alpha . x_i of the hourglass control)
  int hexmean;             // hexahedra: nonzero = uniform gradient, 0 = centre point (Eq. 17)
  double *V;               // [E] exact volume
  double *lamgeo;          // [E] lambda_max(K0_e) / V
  int *nbad;               // inverted / degenerate element count
  int *nnotspd;            // conductivity tensors that are not SPD
  double hg_eps;           // > 0: hourglass control of the uniform-gradient hexahedron
};

struct MassArgs {
  int64_t N;
  int ne;
  const int64_t *inc_ptr;
  const int32_t *inc_elem;
  const MatDev *mats;
  const int32_t *emat;
  const double *ec0;       // nullable, [E]: heat capacity c0 per element (c1 = 0)
  const double *V;
  double T_lo, T_hi;
  double *M0, *M1, *Cmin;  // internal node order
  double fc_min;           // smallest value of the c table on [T_lo, T_hi] (1 without)
};

struct BndArgs {
  int64_t nf;
  int nfn;
  const int32_t *faces;    // caller ids
  const double *x, *y, *z;
  const double *fh, *fTa, *feps, *fq;  // nullable
  double *farea;
  // per boundary record (internal order of the record nodes)
  int64_t nrec;
  const int64_t *rec_ptr;  // CSR over (face id >= 0 | point load -(i+1))
  const int32_t *rec_item;
  const double *pt_W;
  double *bhA, *bhAT, *beA, *bP;
  double *bTa;             // nullable: radiation ambient of the record (the Ta of
                           // its first radiating face), recomputed when given
};

struct DtArgs {
  int ne;
  int64_t E, nrec;
  const double *lamgeo, *kscale;
  const MatDev *mats;
  const int32_t *emat;
  const double *ec0;          // nullable per-element c0 override
  const int32_t *elem_inst;   // nullable
  const int32_t *rec_node;    // internal node of every record
  const int32_t *node_inst;   // nullable, internal order
  const double *bhA, *beA, *Cmin;
  double T_lo, T_hi, Tz;
  unsigned long long *lamE, *lamB;  // per instance, bit patterns of positive doubles
  double fk_max, fc_min;      // extremes of the D and c tables on [T_lo, T_hi] (1 without)
};

struct NodeArrArgs {
  int prec;
  int64_t N, nrec;
  const double *M0, *M1, *dt_inst;
  const int32_t *node_inst;   // nullable
  const uint8_t *is_dir;
  const double *bhA, *bhAT, *beA, *bTa, *bP;
  void *alpha, *beta;         // R[N]
  void *rA, *rAT, *reA, *rTa, *rP;  // R[nrec]
};

// In-run health check (Sec. 3.4: the stability bound holds for temperatures
// in [T_lo, T_hi]): the step kernels record the first step after which a
// temperature left the window or was not finite, and at chosen steps the
// energy balance of the explicit update.  One record per context, written by
// the kernels and read by the host at synchronising calls.
struct Health {
  unsigned long long first_bad;  // smallest step count after which a temperature was
                                 // outside the window or not finite; ~0 = none
  long long base;                // step count at the start of the graph replay in flight
  double energy_max;             // largest relative energy residual of the checks
  long long energy_step;         // step count of that check (-1 = none)
  long long checks;              // energy checks folded
  unsigned int done;             // tiles that have written their partial sums (this check)
  unsigned int pad_;
};

struct StepArgs {
  int prec, ne;
  int k;                      // steps this launch advances (1..tiling depth)
  int tdk, tdc;               // temperature-dependent conductivity / capacity
  int nt, nper, block, lds;
  int pb, maxinc;
  int64_t Eexp;
  const TileHdr *tiles;
  const uint16_t *ent;
  const int32_t *halo;
  const int32_t *rec_of;      // boundary record of an internal node, or -1
  const void *H;
  const void *Tin;
  const float *loin;
  void *Tout;
  float *loout;
  const void *alpha, *beta;
  const void *rA, *rAT, *reA, *rTa, *rP;
  double s0, s1, Tz;
  // conductivity and capacity laws beyond the shared linear ones
  const void *esk;            // nullable R[2][Eexp]: (s0, s1) of each expanded element
  const void *ktab, *ctab;    // nullable R[2 n]: shared multiplier tables of D and c
  int nkt, nct;
  int op;                     // element operator: 0 folded 3x3, 1 uniform-gradient hexahedron
  // health check (nullable hl: none).  The launch's steps are step0 + 1 ..
  // step0 + k (plus hl->base when hbase != 0, in graph replays); energy != 0:
  // the launch's last step is an energy check, each tile adding its partial
  // sums to hpart[tile] and the last tile folding them in tile order
  Health *hl;
  double *hpart;              // [2 nt]
  double win_lo, win_hi;
  float win_lo_f, win_hi_f;   // the window rounded outward to FP32
  long long step0;
  int hbase, energy;
};

// One step of the discrete adjoint of the explicit update.
struct AdjArgs {
  int prec, ne;
  int nt, nper, block, lds;
  int pb, maxinc;
  int64_t Eexp;
  const TileHdr *tiles;
  const uint16_t *ent;
  const int32_t *halo;
  const int32_t *eorig;
  const uint8_t *eowner;
  const void *H;
  const void *alpha;          // R[N]
  const void *rdt;            // R[N]: 1 / dt of the node's instance
  const void *mV;             // R[E]: rho V / n_e of every caller element
  const void *rA;             // R[nrec]: h A of every boundary record
  const void *lamin;          // R[N] lambda^{n+1} (hi)
  const float *lamloin;       // lo part (compensated mode)
  void *lamout;               // lambda^n
  float *lamloout;
  const void *Tn, *Tn1;       // R[N]: T^n and T^{n+1} (hi)
  double *g_logk, *g_c;       // [E] caller element order
  double *S0, *S1;            // [nrec]: sum of mu and of mu T^n
  double s0;
  // temperature dependence: D(T) = Dk s_e when tdk (s_e the element mean of the
  // nodal s0 + s1 T_a, or of the k table's nodal values), capacity
  // alpha + beta T when tdc, radiation sigma eps A per boundary record
  int tdk, tdc;
  double s1, Tz;
  const void *beta;           // R[N]
  const void *reA;            // R[nrec]
  const void *esk, *ktab, *ctab;  // as in StepArgs
  int nkt, nct;
  int op;
};

hipError_t launch_geom(const GeomArgs &a, hipStream_t s);
hipError_t launch_mass(const MassArgs &a, hipStream_t s);
hipError_t launch_bnd(const BndArgs &a, hipStream_t s);
// record powers (face fluxes and concentrated loads, the P of the records that
// launch_bnd derives) for each of nrows rows of point-load values W[nrows][npt],
// cast to the working precision: out[row * nrec + r]
hipError_t launch_point_rows(int prec, const BndArgs &a, int64_t nrows, int64_t npt,
                             const double *W, void *out, hipStream_t s);
hipError_t launch_dt(const DtArgs &a, hipStream_t s);
hipError_t launch_node_arrays(const NodeArrArgs &a, hipStream_t s);
// (s0, s1) of the material of every expanded element, in the step precision
hipError_t launch_expand_sk(int prec, int64_t Eexp, const int32_t *eorig, const MatDev *mats,
                            const int32_t *emat, void *esk, hipStream_t s);
// H = H0 of each expanded element's original (W values), rows >= from scaled by
// the element's conductivity factor
// rows [from, to) of H0 take the per-element conductivity factor
hipError_t launch_expand_H(int prec, int W, int from, int to, int64_t Eexp, int64_t E, const int32_t *eorig,
                           const double *H0, const double *kscale, void *H, hipStream_t s);
// Resident stepping: one launch advances nsteps steps.  Every tile
// keeps its element operators and node coefficients in registers for the whole
// launch.  The temperatures of exported nodes (those in another tile's halo)
// are passed through two exchange buffers of tagged words (FP32: 64 bits, the
// step number and the value; FP64: 16 bytes, step, value, step), so a reader
// polls the data itself until it carries the step it needs.
// largest number of breakpoints of a property table
constexpr int kMaxTablePoints = 16;

struct ResArgs {
  int nsteps;
  int spin_limit;             // polls of a halo word before the wait gives up
  unsigned tag0;              // words written at step s carry tag0 + s + 1
  const uint8_t *exported;    // per internal node: 1 if in another tile's halo
  unsigned long long *X[2];   // exchange buffers, N (FP32) or 2 N (FP64) 64-bit words each
  int *err;                   // set to 1 when a wait gives up
  void *Tfin;                 // final hi (the T buffer of parity cur ^ (nsteps & 1))
  float *lofin;               // final lo (FP32C)
  void *seg;                  // nullable: hi after step s goes to seg + (s + 1) * N (the
                              // adjoint's segment recompute)
  int64_t segN;
  // nullable: per-step record powers R[pts_nrows][pts_nrec]; step s of the launch
  // takes row (pts_row + s) mod pts_nrows in place of rP
  const void *pts;
  int64_t pts_nrec;
  int pts_row, pts_nrows;
  // 1: each step runs the elements whose nodes the tile owns before it waits
  // for the halo (one more workgroup barrier a step); 0: all elements after it
  int split;
  unsigned tag_skew;          // added to the tag a wait looks for: 0, or (tests of the
                              // failure path) a value no word carries
  // table laws: 1 if each step stages the conductivity table's value at every
  // touched node in LDS (the elements average those), 0 if the elements
  // evaluate the table at their nodes
  int nvals;
  // uniform-gradient hexahedron: 1 if the operators of the elements that
  // touch the halo are copied to LDS at the launch's start
  int ophalo;
  // nullable (FP32 hexahedra with the folded operator and the shared laws):
  // per tile, the LDS position of each touched node's temperature and slots,
  // at [tile * sstride + local index]: the tile's touched nodes in caller
  // order, so a wave's elements gather and scatter mostly consecutive LDS
  // words; null: the local index itself
  const int16_t *sigma;
  int sstride;
  const void *ent_sigma;  // with sigma: the packed entries with those positions
};

// Resident adjoint of one checkpoint segment (hexahedra, folded operator):
// nsteps adjoint steps over the stored states T^{n0 + i} at seg + i * segN,
// i = 0..nsteps, with the exchange of ResArgs.
struct AdjResArgs {
  int nsteps;
  int spin_limit;
  unsigned tag0;
  const uint8_t *exported;
  unsigned long long *X[2];
  int *err;
  const void *seg;
  int64_t segN;
};

// register capacity of the resident kernel per thread (elements, nodes, halo ids)
struct ResCaps {
  int ept, npt, hpt;
};
ResCaps resident_caps(int prec, int ne);
hipError_t launch_step(const StepArgs &a, hipStream_t s);
hipError_t launch_resident(const StepArgs &a, const ResArgs &r, hipStream_t s);
// LDS limit of the resident kernel; *blocks_per_cu receives how many of its
// workgroups of a.block threads one CU holds at once
hipError_t resident_prepare(const StepArgs &a, int *blocks_per_cu);
hipError_t step_set_lds_limit(int prec, int ne, int tdk, int tdc, int gen, int op, int bytes);
hipError_t launch_adjoint(const AdjArgs &a, hipStream_t s);
// gen: the instance for property tables (else the linear laws only)
hipError_t adjres_prepare(int prec, int gen, int block, int lds, int *blocks_per_cu);
hipError_t launch_adjres(const AdjArgs &a, const AdjResArgs &r, hipStream_t s);
hipError_t adjoint_set_lds_limit(int prec, int ne, int op, int bytes);
// g_h[f] = -|f|/n_f * sum over the face's nodes of (S1 - Ta_f S0)
hipError_t launch_face_grad(int64_t nf, int nfn, const int32_t *faces, const int32_t *perm,
                            const int32_t *rec_of, const double *farea, const double *fTa,
                            const double *S0, const double *S1, double *g_h, hipStream_t s);
// 1 / dt per internal node and rho V / n_e per caller element
hipError_t launch_adjoint_coefs(int prec, int64_t N, int64_t E, int ne, const double *dt_inst,
                                const int32_t *node_inst, const MatDev *mats,
                                const int32_t *emat, const double *V, void *rdt, void *mV,
                                hipStream_t s);

// caller-order FP64 temperatures <-> internal working arrays
hipError_t launch_set_T(int prec, int64_t N, const double *Tuser, const int32_t *perm,
                        void *T, float *lo, int64_t ndir, const int32_t *dir_node,
                        const double *dir_T, hipStream_t s);
hipError_t launch_get_T(int prec, int64_t N, const int32_t *perm, const void *T,
                        const float *lo, double *Tuser, hipStream_t s);
hipError_t launch_check(int prec, int64_t N, const void *T, const float *lo, double lo_b,
                        double hi_b, int *flag, hipStream_t s);
// health record: op 0 reset (no bad step, no checks, base = 0), op 1 set the
// graph replays' base step count to v, op 2 advance it by v, op 3 clear the
// out-of-window record
hipError_t launch_health(Health *h, int op, long long v, hipStream_t s);
// gather/scatter of raw working arrays between caller and internal order
// smallest / largest temperature as order keys (keys[0] must start at ~0,
// keys[1] at 0); *nan |= 1 if a temperature is not finite
hipError_t launch_range(int prec, int64_t N, const void *T, const float *lo,
                        unsigned long long *keys, int *nan, hipStream_t s);
hipError_t launch_permute(int elem_bytes, int64_t N, const int32_t *perm, const void *src,
                          void *dst, int to_internal, hipStream_t s);

// Device address of the static scratch array on the current device (looked up
// once per device); it holds kScratchBytes bytes.
constexpr size_t kScratchBytes = FED_NOALLOC_SCRATCH_BYTES;
hipError_t scratch_address(void **ptr);

}  // namespace fed
