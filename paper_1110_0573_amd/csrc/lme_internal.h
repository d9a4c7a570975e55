// lme_internal.h -- data layout shared by the host planner and the gfx950
// kernels of the Lindblad library.  Not part of the public ABI.
//
// Operator form of the Liouvillian (Eq. (master_equation), hbar = 1):
//   L y = A y + y A^+ + sum_k C_k y C_k^+ ,   A = -i H - 1/2 sum_k C_k^+ C_k,
// with H = H0 + sum_j u_j H_j, so A = A0 + sum_j u_j B_j, B_j = -i H_j.
// The adjoint L^+ x = A^+ x + x A + sum_k C_k^+ x C_k has the same shape with
// (A, B_j, C_k) replaced by (A^+, B_j^+, C_k^+); one kernel serves both.
//
// Each instance's operators are packed into one byte blob ("op blob") that a
// workgroup copies verbatim into LDS:
//   D     [n]          complex  diagonal of A0
//   Oval  [wo][n]      complex  off-diagonal entries of A0, ELL, slot-major
//   Ocol  [wo][n]      int32    their columns (padding: col = row, val = 0)
//   Jval  [nc][wc][n]  complex  every entry of C_k, ELL
//   Jcol  [nc][wc][n]  int32
//   DB    [nb][n]      complex  diagonal of B_j
//   OBval [nb][wb][n]  complex  off-diagonal of B_j, ELL
//   OBcol [nb][wb][n]  int32
// Sections start on 16-byte boundaries.  ELL slot-major order puts rows i and
// i+1 of one slot next to each other, so a wave reading consecutive rows
// reads consecutive addresses.
#pragma once
#include <math.h>
#include <stdint.h>

#ifdef __HIPCC__
#define LME_HD __host__ __device__
#else
#define LME_HD
#endif

namespace lme {

constexpr int kMaxWidth = 64;       // max non-zeros per operator row
constexpr int kMaxDim = 4096;
constexpr int kMaxPack = 1023;   // instances per resident pack (10-bit slot field)

LME_HD inline int32_t align16(int32_t x) { return (x + 15) & ~15; }

struct BlobLayout {
  int32_t n, wo, nb, wb, nc, wc;
  int32_t offD, offOval, offOcol, offJval, offJcol, offDB, offOBval, offOBcol;
  int32_t bytes;
};

LME_HD inline BlobLayout blob_layout(int32_t n, int32_t wo, int32_t nb, int32_t wb,
                                     int32_t nc, int32_t wc) {
  BlobLayout L;
  L.n = n; L.wo = wo; L.nb = nb; L.wb = wb; L.nc = nc; L.wc = wc;
  int32_t o = 0;
  L.offD = o;     o = align16(o + 16 * n);
  L.offOval = o;  o = align16(o + 16 * wo * n);
  L.offOcol = o;  o = align16(o + 4 * wo * n);
  L.offJval = o;  o = align16(o + 16 * nc * wc * n);
  L.offJcol = o;  o = align16(o + 4 * nc * wc * n);
  L.offDB = o;    o = align16(o + 16 * nb * n);
  L.offOBval = o; o = align16(o + 16 * nb * wb * n);
  L.offOBcol = o; o = align16(o + 4 * nb * wb * n);
  L.bytes = o;
  return L;
}

// Expectation operators of one instance: Ecol[m][we][n] int32 then
// Eval[m][we][n] complex (ELL of every entry, padding val = 0, col = row).
LME_HD inline int64_t eops_val_offset(int32_t n, int32_t we, int32_t n_e) {
  return align16(4 * n_e * we * n);
}
LME_HD inline int64_t eops_bytes(int32_t n, int32_t we, int32_t n_e) {
  return eops_val_offset(n, we, n_e) + 16LL * n_e * we * n;
}

// Operator signature: instances sharing it have identically laid-out blobs.
struct Signature {
  int32_t n, wo, nb, wb, nc, wc;
};

// Value-structure flags of an instance's forward operators.
enum : int32_t {
  kJumpsReal = 1,         // every collapse-operator entry is real
  kOffdiagImag = 2,       // off-diagonal entries of A and of every -iH_j are imaginary
};

struct InstDesc {
  int64_t rho_off;    // complex elements into the packed state
  int64_t ops_off;    // bytes into the forward op pool
  int64_t adj_off;    // bytes into the adjoint op pool
  int64_t eops_off;   // bytes into the expectation-op pool
  int32_t n, we;      // dimension, expectation-op ELL width
  Signature fwd, adj;
  int32_t fwd_bytes, adj_bytes;
  int32_t flags;      // kJumpsReal | kOffdiagImag
};

// A pack: m instances with one signature, integrated by one workgroup.
struct PackDesc {
  int32_t first;      // index into the instance order array
  int32_t m;          // instances in the pack
  int32_t n, wo, nb, wb, nc, wc;
  int32_t blob_bytes; // per instance
  int32_t lds_bytes;  // total dynamic LDS this pack needs
  int32_t G;          // column-owner kernels: row groups (threads per column)
  int32_t ept;        // column-owner kernels: rows per thread, ceil(n / G)
  int32_t awo, awb, awc;  // gradient kernel: widths of the adjoint blob
  int32_t fwd_bytes;      // gradient kernel: forward part of blob_bytes
  int32_t blob_stride;    // LDS distance between consecutive instances' blobs
  int32_t pad_;
};

// Column-owner kernels hold one column's operator entries in registers; they
// take operators with at most these widths (monomial jumps).
constexpr int kColWO = 2;   // off-diagonal entries per row of A
constexpr int kColNC = 3;   // collapse operators
constexpr int kColWB = 2;   // off-diagonal entries per row of a control term
// (threads per workgroup, rows per thread) of the column-owner kernels
constexpr int kColCfg[2][2] = {{512, 14}, {768, 9}};
// Hermitian column-owner configurations (about half the rows per column)
constexpr int kHermCfg[2][2] = {{512, 8}, {768, 5}};

// The Hermitian RK4 kernel keeps each slot's row data in registers (and no
// operator data in LDS) for real structure with at most 3 monomial operator
// columns per row and no control terms; otherwise it reads row records.
LME_HD constexpr bool herm_slots(bool re, int32_t wo, int32_t nc, int32_t nb) {
  return re && nb == 0 && wo + nc <= 3;
}

// Row records of the column-owner kernels (one per operator row, in LDS):
// 1 + wo + nc + nb*kColWB int32 byte offsets, padded to 16 bytes, then
// 1 + wo + nc + nb*(1 + kColWB) complex coefficients; the record is an odd
// number of 16-byte units.
LME_HD constexpr int32_t rec_hdr_bytes(int32_t wo, int32_t nc, int32_t nb) {
  return (4 * (1 + wo + nc + nb * kColWB) + 15) & ~15;
}
LME_HD constexpr int32_t rec_bytes(int32_t wo, int32_t nc, int32_t nb) {
  return rec_hdr_bytes(wo, nc, nb) + 16 * (1 + wo + nc + nb * (1 + kColWB)) +
         ((((rec_hdr_bytes(wo, nc, nb) / 16) + 1 + wo + nc + nb * (1 + kColWB)) & 1) ? 0 : 16);
}

// Per-call arguments of the resident RK4 kernel.
struct Rk4Args {
  const PackDesc *packs;
  const int32_t *order;     // pack slot -> instance index
  const InstDesc *inst;
  const uint8_t *ops;       // op pool (forward or adjoint)
  int32_t adjoint;          // use adj_off instead of ops_off
  const uint8_t *eops;
  const double *u;          // [n_inst][n_ctrl][n_seg] or null
  int32_t n_ctrl, n_seg, n_e, n_t;
  const int32_t *seg_of_step;  // [nsteps] segment index or -1
  const int32_t *out_step;     // [n_t] step index after which output k is due
  int32_t nsteps;
  double h;
  const double *fn;         // [n_inst][n_ctrl][7] closed-form amplitudes or null
  double t0;                // time of step 0 (closed-form amplitudes)
  int64_t state_elems;
  const double *rho0;       // complex128 packed (interleaved)
  double *rho_out;
  double *states;           // [n_t][state_elems]
  double *expect;           // [n_inst][n_e][n_t]
  int64_t *counts;          // [n_inst][2]
  int32_t *status;          // [n_inst]
};

// Closed-form amplitude c0 + c1 t + c2 t^2 + c3 t^3 + a cos(w t + phi) with
// p = (c0, c1, c2, c3, a, w, phi).
LME_HD inline double coeff_fn_at(const double *p, double t) {
  // without a cosine term the polynomial alone (the cosine's product with a
  // zero amplitude could only change the sign of a zero result)
  const double poly = p[0] + t * (p[1] + t * (p[2] + t * p[3]));
  return p[4] != 0.0 ? poly + p[4] * cos(p[5] * t + p[6]) : poly + 0.0;
}

// Monte-Carlo wave-function kernel (lme_mc.hip).  Operators of one system:
// A = -i H - 1/2 sum_n C_n^+ C_n as diagonal D[n] plus ELL off-diagonal
// Oval/Ocol[wo][n]; collapse operators Jval/Jcol[nc][wc][n]; expectation
// operators Eval/Ecol[ne][we][n] (ELL padding: value 0, column = row).
constexpr int kMcMaxNC = 16;     // collapse operators
constexpr int kMcMaxDim = 8192;  // largest dimension (the kernel's row capacity)

struct McLayout {
  int64_t offD, offOval, offOcol, offJval, offJcol, offEval, offEcol, bytes;
};

LME_HD inline McLayout mc_layout(int32_t n, int32_t wo, int32_t nc, int32_t wc, int32_t ne,
                                 int32_t we) {
  McLayout L;
  int64_t o = 0;
  auto al = [](int64_t x) { return (x + 255) & ~int64_t(255); };
  L.offD = o;    o = al(o + 16LL * n);
  L.offOval = o; o = al(o + 16LL * wo * n);
  L.offOcol = o; o = al(o + 4LL * wo * n);
  L.offJval = o; o = al(o + 16LL * nc * wc * n);
  L.offJcol = o; o = al(o + 4LL * nc * wc * n);
  L.offEval = o; o = al(o + 16LL * ne * we * n);
  L.offEcol = o; o = al(o + 4LL * ne * we * n);
  L.bytes = o;
  return L;
}

struct McArgs {
  int32_t n, wo, nc, wc, ne, we;
  int32_t G, P;                 // threads per trajectory (2^k), trajectories per workgroup
  int32_t n_traj, n_t, nsteps, max_jumps;
  double t0, h;
  const double *D, *Oval, *Jval, *Eval;   // complex128
  const int32_t *Ocol, *Jcol, *Ecol;
  const int32_t *out_step;      // [n_t]: grid step after which output k is due
  const double *psi0;           // complex128 [n]
  const double *draws;          // [n_traj][max_jumps + 1][2]
  double *ex_traj;              // complex128 [n_traj][ne][n_t]
  int32_t *n_jumps;             // [n_traj] or null
  double *jump_t;               // [n_traj][max_jumps] or null
  int32_t *jump_op;             // [n_traj][max_jumps] or null
  int32_t *status;              // [n_traj] or null
  double *vbuf;                 // complex128 [gridDim][4][P][n]: Taylor vectors of a jump
};

// Per-call arguments of the resident Dormand-Prince kernel.
struct Dp5Args {
  const PackDesc *packs;
  const int32_t *order;
  const InstDesc *inst;
  const uint8_t *ops;
  const uint8_t *eops;
  const double *u;          // [n_inst][n_ctrl][n_seg] or null
  int32_t n_ctrl, n_seg, n_e, n_t;
  const double *stops;      // [n_stops] stop times after t0 (outputs, edges)
  const int32_t *stop_out;  // [n_stops] output index landed on, or -1
  const int32_t *stop_seg;  // [n_stops] control segment of the interval ending there
  int32_t n_stops;
  double t0, rtol, atol, h0, h_min;
  int64_t max_steps;
  int64_t state_elems;
  double *kbuf;             // [7][state_elems] complex: stage derivatives
  const double *rho0;
  double *rho_out;
  double *states;           // [n_t][state_elems]
  double *expect;           // [n_inst][n_e][n_t]
  int64_t *counts;          // [n_inst][2]
  int32_t *status;          // [n_inst]
};

// Per-call arguments of the resident cost-gradient kernel.
constexpr int kMaxGradCtrl = 4;
struct GradArgs {
  const PackDesc *packs;    // packs over the forward signature
  const int32_t *order;
  const InstDesc *inst;
  const uint8_t *ops;       // forward op pool
  const uint8_t *adj;       // adjoint op pool
  const double *u;          // [n_inst][n_ctrl][n_seg]
  int32_t n_ctrl, n_seg;
  const int32_t *seg_of_step;  // [nsteps]
  int32_t nsteps, ckpt_every;
  double h;
  int64_t state_elems;
  const double *rho0;
  const double *O;          // packed like the states
  double *ckpt;             // [n_ckpt][state_elems] complex
  double *stages;           // [ckpt_every][4][state_elems] complex
  double *cost;             // [n_inst]
  double *grad;             // [n_inst][n_ctrl][n_seg]
};

// A streamed tile: elements [e0, e1) of instance `inst`.
struct Tile {
  int32_t inst, e0, e1, pad;
};

// Per-call arguments of the streamed (HBM-resident) Liouvillian application:
// out[b] = L_b(t) y[b] for every tile.
struct ApplyGArgs {
  const Tile *tiles;
  int32_t n_tiles;
  const InstDesc *inst;
  const uint8_t *ops;
  int32_t adjoint;
  const double *u;
  int32_t n_ctrl, n_seg, seg;
  const double *y;
  double *out;
};

// Superoperator SpMV: per instance an ELL matrix of n^2 rows, width w,
// slot-major: col[s * n^2 + e], val[s * n^2 + e].
struct SuperDesc {
  int64_t col_off;    // int32 elements into the column pool
  int64_t val_off;    // complex elements into the value pool
  int32_t w, pad;
};

struct SuperArgs {
  const Tile *tiles;
  int32_t n_tiles;
  const InstDesc *inst;
  const SuperDesc *sd;
  const int32_t *col;
  const double *val;
  const double *y;
  double *out;
};

// Per-instance adaptive step control (LDS in the resident kernel, HBM in the
// streamed one).
struct DpCtl {
  double t, h, h_try, hs;
  int64_t n_acc, n_rej;
  int32_t stop, status, active, accept, landing, seg, k1_seg, prev_rej, out_due, need_k1;
};

// Per-call arguments of the streamed steppers (one grid-wide kernel per
// stage; state and stage data in HBM).
struct StreamArgs {
  const Tile *tiles;
  int32_t n_tiles, n_inst;
  const int32_t *tile_first;   // [n_inst] first tile of each instance
  const int32_t *tile_count;   // [n_inst]
  const InstDesc *inst;
  const uint8_t *ops;
  const uint8_t *eops;
  const double *u;
  int32_t n_ctrl, n_seg, n_e, n_t;
  int64_t state_elems;
  double *rho, *yb0, *yb1, *y5, *acc;
  double *K;                   // [7][state_elems]
  double *tile_part;           // [2 n_tiles]
  // adaptive
  DpCtl *ctl;
  const double *stops;
  const int32_t *stop_out, *stop_seg;
  int32_t n_stops;
  double t0, rtol, atol, h0, h_min;
  int64_t max_steps;
  int32_t *n_active;           // written by the control kernel
  // fixed step
  const int32_t *seg_of_step, *out_step;
  int32_t nsteps;
  double h;
  int32_t *counters;           // [0] completed steps, [1] next output
  // outputs
  double *states, *expect;
  int64_t *counts;
  int32_t *status;
};

// Per-call arguments of the one-shot Liouvillian application.
struct ApplyArgs {
  const PackDesc *packs;
  const int32_t *order;
  const InstDesc *inst;
  const uint8_t *ops;
  int32_t adjoint;
  const double *u;
  int32_t n_ctrl, n_seg, seg;
  const double *y;
  double *out;
};

// Pipelined column application.  A tile is either m whole instances of one
// signature (r0 = h0 = 0, r1 = span = n) or rows [r0, r1) of one instance
// together with the rows [h0, h0 + span) its products read (a band around
// them).  Each buffer of the workgroup's two LDS stages holds the tile's y
// rows and the row records of all its instances' rows.
constexpr int kPipeT = 1024;          // threads per workgroup
constexpr int kPipeStage = 71680;     // bytes per LDS stage (y + records)
constexpr int kPipeUnits = (kPipeStage / 16 + kPipeT - 1) / kPipeT;  // 16-B loads per thread
constexpr int kPipeMaxM = 8;          // instances per tile
constexpr int kPipeMaxTiles = 64;     // tiles per workgroup (descriptors kept in LDS)
constexpr int kPipeEPT = 8;           // rows per thread of a tile

struct PTile {
  int32_t m, n, G;  // instances, dimension, row groups
  int32_t r0, r1;   // rows computed
  int32_t h0, span; // rows staged: [h0, h0 + span) of each instance
  int32_t wb;       // control-term width of the signature
  int32_t rec_lds;  // byte offset of the records in the stage buffer
  int32_t pad[3];
  int64_t yoff[kPipeMaxM];  // state offset of each instance (elements)
  int64_t roff[kPipeMaxM];  // record offset of each instance (bytes)
  int32_t id[kPipeMaxM];    // instance index
};

struct PipeArgs {
  const PTile *tiles;
  int32_t n_tiles;
  const uint8_t *recs;   // row records of every instance (HBM)
  const double *u;
  int32_t n_ctrl, n_seg, seg;
  const double *y;
  double *out;
};

}  // namespace lme
