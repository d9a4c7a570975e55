// lme_kernels.hip -- gfx950 kernels of the Lindblad library.
//
// All arithmetic is FP64 complex.  The Liouvillian is applied in operator
// form (Eq. (master_equation), hbar = 1):
//   k_ij = (A y + y A^+ + sum_k C_k y C_k^+)_ij
//        = (D_i + conj(D_j)) y_ij
//          + sum_w O_iw y[col_iw][j] + sum_w conj(O_jw) y[i][col_jw]
//          + sum_q u_q (same three terms for B_q = -i H_q)
//          + sum_k sum_{w,v} J_kiw conj(J_kjv) y[col_kiw][col_kjv]
// where A = D + O (diagonal + off-diagonal ELL).  Every term is a gather from
// the stage input y, which the resident kernels keep in LDS.
#include <hip/hip_runtime.h>

#include "lme_internal.h"

namespace lme {

// ---------------------------------------------------------------------------
// complex helpers (double2 = re, im)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// a * b with the product fused into each sum written out: left to the
// compiler, which product of a.x b.y + a.y b.x it fuses depends on the
// surrounding code, and two kernels evaluating the same element could round
// it differently
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
// c + a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
// c + conj(a) * b
__device__ __forceinline__ double2 cfma_conj(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y)));
}
// c + s * a  (s real)
__device__ __forceinline__ double2 caxpy(double s, double2 a, double2 c) {
  return make_double2(fma(s, a.x, c.x), fma(s, a.y, c.y));
}
__device__ __forceinline__ bool cfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// ---------------------------------------------------------------------------
// operator view of one instance's op blob
// ---------------------------------------------------------------------------
struct OpView {
  const double2 *D, *Oval, *Jval, *DB, *OBval;
  const int32_t *Ocol, *Jcol, *OBcol;
  int n, wo, nb, wb, nc, wc;
};

__device__ __forceinline__ OpView make_view(const uint8_t *blob, const BlobLayout &L) {
  OpView v;
  v.D = reinterpret_cast<const double2 *>(blob + L.offD);
  v.Oval = reinterpret_cast<const double2 *>(blob + L.offOval);
  v.Ocol = reinterpret_cast<const int32_t *>(blob + L.offOcol);
  v.Jval = reinterpret_cast<const double2 *>(blob + L.offJval);
  v.Jcol = reinterpret_cast<const int32_t *>(blob + L.offJcol);
  v.DB = reinterpret_cast<const double2 *>(blob + L.offDB);
  v.OBval = reinterpret_cast<const double2 *>(blob + L.offOBval);
  v.OBcol = reinterpret_cast<const int32_t *>(blob + L.offOBcol);
  v.n = L.n; v.wo = L.wo; v.nb = L.nb; v.wb = L.wb; v.nc = L.nc; v.wc = L.wc;
  return v;
}

// (A y + y A^+)_ij restricted to a diagonal + ELL operator (D, Oval, Ocol).
__device__ __forceinline__ double2 two_sided(const double2 *D, const double2 *Oval,
                                             const int32_t *Ocol, int wo, int n,
                                             const double2 *Y, int i, int j, double2 yij) {
  double2 acc = cmul(cadd(D[i], cconj(D[j])), yij);
  for (int w = 0; w < wo; ++w) {
    const int c = Ocol[w * n + i];
    acc = cfma(Oval[w * n + i], Y[c * n + j], acc);
  }
  for (int w = 0; w < wo; ++w) {
    const int c = Ocol[w * n + j];
    acc = cfma_conj(Oval[w * n + j], Y[i * n + c], acc);
  }
  return acc;
}

// Element (i, j) of L y for one instance; Y is that instance's n x n stage
// input, uq[q * ustride] its nb control amplitudes for the current step.
__device__ __forceinline__ double2 lindblad_elem(const OpView &op, const double2 *Y,
                                                 int i, int j, double2 yij,
                                                 const double *uq, int ustride = 1) {
  const int n = op.n;
  double2 acc = two_sided(op.D, op.Oval, op.Ocol, op.wo, n, Y, i, j, yij);
  for (int q = 0; q < op.nb; ++q) {
    const double u = uq[q * ustride];
    if (u != 0.0) {
      const double2 t = two_sided(op.DB + q * n, op.OBval + q * op.wb * n,
                                  op.OBcol + q * op.wb * n, op.wb, n, Y, i, j, yij);
      acc = caxpy(u, t, acc);
    }
  }
  for (int k = 0; k < op.nc; ++k) {
    const double2 *Jv = op.Jval + k * op.wc * n;
    const int32_t *Jc = op.Jcol + k * op.wc * n;
    for (int w = 0; w < op.wc; ++w) {
      const double2 vi = Jv[w * n + i];
      const int ci = Jc[w * n + i];
      for (int v = 0; v < op.wc; ++v) {
        const double2 p = cmul(vi, cconj(Jv[v * n + j]));
        acc = cfma(p, Y[ci * n + Jc[v * n + j]], acc);
      }
    }
  }
  return acc;
}

// Copies the m op blobs of a pack into LDS (16-byte vector copies).
__device__ __forceinline__ void stage_blobs(uint8_t *dst, const PackDesc &pk,
                                            const int32_t *order, const InstDesc *inst,
                                            const uint8_t *pool, int adjoint) {
  const int nvec = pk.blob_bytes / 16;
  const int total = pk.m * nvec;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int b = idx / nvec, r = idx - b * nvec;
    const InstDesc &d = inst[order[pk.first + b]];
    const uint4 *src = reinterpret_cast<const uint4 *>(pool + (adjoint ? d.adj_off : d.ops_off));
    reinterpret_cast<uint4 *>(dst + (size_t)b * pk.blob_stride)[r] = src[r];
  }
}

// Deterministic butterfly sum over the 64 lanes of a wavefront.
__device__ __forceinline__ double2 wave_sum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// LDS carve-up of a pack:
//   Y [E] | blobs [m][blob_bytes] | u [m][nb] | state offsets [m] | ids [m]
struct PackLds {
  double2 *Y;
  uint8_t *blobs;
  double *u;
  int64_t *off;
  int32_t *ids;
};

// LDS stride between the op blobs of a pack: an odd number of 16-byte units,
// so that the lanes of one wave reading the same row of different instances
// fall into different LDS banks.
__host__ __device__ inline int32_t blob_stride_of(int32_t blob_bytes) {
  return ((blob_bytes / 16) & 1) ? blob_bytes : blob_bytes + 16;
}

__host__ __device__ inline int32_t pack_lds_bytes(int32_t n, int32_t m, int32_t blob_bytes,
                                                  int32_t nb) {
  return align16(16 * m * n * n) + m * blob_stride_of(blob_bytes) + align16(8 * m * nb) +
         align16(8 * m) + align16(4 * m);
}

__device__ __forceinline__ PackLds carve(uint8_t *smem, const PackDesc &pk) {
  PackLds p;
  const int E = pk.m * pk.n * pk.n;
  p.Y = reinterpret_cast<double2 *>(smem);
  p.blobs = smem + align16(16 * E);
  p.u = reinterpret_cast<double *>(p.blobs + (size_t)pk.m * pk.blob_stride);
  p.off = reinterpret_cast<int64_t *>(reinterpret_cast<uint8_t *>(p.u) + align16(8 * pk.m * pk.nb));
  p.ids = reinterpret_cast<int32_t *>(reinterpret_cast<uint8_t *>(p.off) + align16(8 * pk.m));
  return p;
}

// Slot coordinates packed in one register: instance-in-pack (10 bits), row
// and column (11 bits each).  Resident packs hold at most 8192 elements.
__device__ __forceinline__ uint32_t pack_bij(int b, int i, int j) {
  return ((uint32_t)b << 22) | ((uint32_t)i << 11) | (uint32_t)j;
}
__device__ __forceinline__ int slot_b(uint32_t v) { return (int)(v >> 22); }
__device__ __forceinline__ int slot_i(uint32_t v) { return (int)((v >> 11) & 2047u); }
__device__ __forceinline__ int slot_j(uint32_t v) { return (int)(v & 2047u); }

// ---------------------------------------------------------------------------
// Resident fixed-step RK4: one workgroup integrates one pack for all steps.
// Thread t owns pack elements f = t + s*T (s < EPT); its rho, the RK4
// accumulator and the next stage input stay in VGPRs; the current stage
// input is shared through LDS.  Two barriers per stage, none across
// workgroups.
// ---------------------------------------------------------------------------
template <int T>
__device__ void write_outputs(const Rk4Args &a, const PackDesc &pk, const PackLds &L,
                              int k) {
  const int n = pk.n, n2 = n * n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ntask = pk.m * a.n_e;
  for (int task = wave; task < ntask; task += T / 64) {
    const int b = task / a.n_e, e = task - b * a.n_e;
    const int id = L.ids[b];
    const InstDesc &d = a.inst[id];
    const int we = d.we;
    const int32_t *Ec = reinterpret_cast<const int32_t *>(a.eops + d.eops_off);
    const double2 *Ev = reinterpret_cast<const double2 *>(
        a.eops + d.eops_off + eops_val_offset(n, we, a.n_e));
    const double2 *Y = L.Y + b * n2;
    double2 part = make_double2(0.0, 0.0);
    for (int i = lane; i < n; i += 64)
      for (int w = 0; w < we; ++w) {
        const int idx = (e * we + w) * n + i;
        part = cfma(Ev[idx], Y[Ec[idx] * n + i], part);
      }
    part = wave_sum(part);
    if (lane == 0) {
      double *dst = a.expect + 2 * (((int64_t)id * a.n_e + e) * a.n_t + k);
      dst[0] = part.x;
      dst[1] = part.y;
      if (!cfinite(part) && a.status) a.status[id] = 5;  // LME_ENONFINITE
    }
  }
}

// Amplitudes of stage `stage` (0..3) of RK4 step st: the segment values
// (the same for every stage) or, with closed-form amplitudes, their values at
// the stage's time t, t + h/2, t + h/2, t + h.  One thread per (instance,
// term) of the pack; the caller synchronises.
__device__ __forceinline__ void rk4_stage_controls(const Rk4Args &a, const PackDesc &pk,
                                                   const int32_t *ids, double *u, int st,
                                                   int stage, int tid, int T) {
  const double tb = a.t0 + (double)st * a.h;
  const double ts = stage == 0 ? tb : (stage == 3 ? tb + a.h : tb + 0.5 * a.h);
  const int seg = a.seg_of_step[st];
  for (int idx = tid; idx < pk.m * pk.nb; idx += T) {
    const int b = idx / pk.nb, q = idx - b * pk.nb;
    const int64_t c = (int64_t)ids[b] * a.n_ctrl + q;
    u[idx] = a.fn ? coeff_fn_at(a.fn + 7 * c, ts) : (seg >= 0 ? a.u[c * a.n_seg + seg] : 0.0);
  }
}

template <int T, int EPT>
__global__ __launch_bounds__(T) void rk4_resident_kernel(Rk4Args a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const PackDesc pk = a.packs[blockIdx.x];
  const int n = pk.n, n2 = n * n, E = pk.m * n2;
  const PackLds L = carve(smem, pk);
  const BlobLayout BL = blob_layout(n, pk.wo, pk.nb, pk.wb, pk.nc, pk.wc);
  const int tid = threadIdx.x;

  for (int b = tid; b < pk.m; b += T) {
    const int id = a.order[pk.first + b];
    L.ids[b] = id;
    L.off[b] = a.inst[id].rho_off;
    if (a.status) a.status[id] = 0;
  }
  stage_blobs(L.blobs, pk, a.order, a.inst, a.ops, a.adjoint);
  __syncthreads();
  // closed-form amplitudes with one (instance, term) pair per thread: the
  // pair's seven coefficients are read once into registers, so a stage's
  // amplitudes wait on no memory load
  const bool fn_reg = a.fn != nullptr && pk.m * pk.nb <= T;
  double cf[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) cf[k] = 0.0;
  if (fn_reg && tid < pk.m * pk.nb) {
    const int b = tid / pk.nb, q = tid - b * pk.nb;
    const double *p = a.fn + 7 * ((int64_t)L.ids[b] * a.n_ctrl + q);
#pragma unroll
    for (int k = 0; k < 7; ++k) cf[k] = p[k];
  }

  double2 rho[EPT], acc[EPT], yn[EPT];
  uint32_t bij[EPT];
  const double2 *rho0 = reinterpret_cast<const double2 *>(a.rho0);
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int f = tid + s * T;
    rho[s] = make_double2(0.0, 0.0);
    bij[s] = 0;
    if (f < E) {
      const int b = f / n2, r = f - b * n2;
      const int i = r / n;
      bij[s] = pack_bij(b, i, r - i * n);
      rho[s] = rho0[L.off[b] + r];
    }
  }

  const bool want_expect = a.expect != nullptr && a.n_e > 0;
  int next_out = 0;
  const double h = a.h;
  for (int st = 0;; ++st) {
    // outputs due after st steps (st = 0: the initial state)
    while (next_out < a.n_t && a.out_step[next_out] == st) {
      __syncthreads();
#pragma unroll
      for (int s = 0; s < EPT; ++s) {
        const int f = tid + s * T;
        if (f < E) {
          L.Y[f] = rho[s];
          if (a.states) {
            const uint32_t v = bij[s];
            const int64_t g = L.off[slot_b(v)] + slot_i(v) * n + slot_j(v);
            reinterpret_cast<double2 *>(a.states)[(int64_t)next_out * a.state_elems + g] = rho[s];
          }
        }
      }
      __syncthreads();
      if (want_expect) write_outputs<T>(a, pk, L, next_out);
      ++next_out;
    }
    if (st == a.nsteps) break;

#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      yn[s] = rho[s];
      acc[s] = make_double2(0.0, 0.0);
    }
    for (int stage = 0; stage < 4; ++stage) {
      // RK4 tableau: stage inputs rho + c*h*k_prev, weights 1, 2, 2, 1
      const double cnext = stage < 2 ? 0.5 * h : (stage == 2 ? h : 0.0);
      const double wgt = (stage == 0 || stage == 3) ? 1.0 : 2.0;
      __syncthreads();  // every reader of the previous stage input is done
      if (fn_reg) {
        if (tid < pk.m * pk.nb) {  // the times of rk4_stage_controls()
          const double tb = a.t0 + (double)st * a.h;
          const double ts = stage == 0 ? tb : (stage == 3 ? tb + a.h : tb + 0.5 * a.h);
          L.u[tid] = coeff_fn_at(cf, ts);
        }
      } else if (pk.nb > 0 && (stage == 0 || a.fn)) {
        rk4_stage_controls(a, pk, L.ids, L.u, st, stage, tid, T);
      }
#pragma unroll
      for (int s = 0; s < EPT; ++s) {
        const int f = tid + s * T;
        if (f < E) L.Y[f] = yn[s];
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < EPT; ++s) {
        const int f = tid + s * T;
        if (f < E) {
          uint32_t v = bij[s];
          // opaque to the optimiser: stops per-slot addresses from being
          // hoisted out of the step loop (which costs ~20 VGPRs per slot)
          asm volatile("" : "+v"(v));
          const int b = slot_b(v);
          const OpView op = make_view(L.blobs + (size_t)b * pk.blob_stride, BL);
          const double2 kv =
              lindblad_elem(op, L.Y + b * n2, slot_i(v), slot_j(v), yn[s], L.u + b * pk.nb);
          acc[s] = caxpy(wgt, kv, acc[s]);
          yn[s] = caxpy(cnext, kv, rho[s]);
        }
        // keep one slot's temporaries live at a time
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int s = 0; s < EPT; ++s) rho[s] = caxpy(h / 6.0, acc[s], rho[s]);
  }

  if (a.rho_out) {
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int f = tid + s * T;
      if (f < E) {
        const uint32_t v = bij[s];
        reinterpret_cast<double2 *>(a.rho_out)[L.off[slot_b(v)] + slot_i(v) * n + slot_j(v)] =
            rho[s];
      }
    }
  }
  if (a.counts)
    for (int b = tid; b < pk.m; b += T) {
      a.counts[2 * (int64_t)L.ids[b]] = a.nsteps;
      a.counts[2 * (int64_t)L.ids[b] + 1] = 0;
    }
}

// ---------------------------------------------------------------------------
// Resident fixed-step RK4 for small instances (n^2 <= 64): one wavefront per
// pack, one element per lane, an instance's elements in consecutive lanes.
// Each lane keeps its element's operator terms in registers (coefficients and
// the lanes of their sources, in the order of lindblad_elem()) and reads the
// stage input of its instance from the other lanes with cross-lane permutes,
// so a stage touches no LDS and needs no barrier.  The terms are those of
// lindblad_elem() in its order, so the results have the bits of
// rk4_resident_kernel.
// Operator widths: at most kLaneWO off-diagonals per row of A, kLaneNB
// control terms of kLaneWB off-diagonals, kLaneJ jump products per element.
// ---------------------------------------------------------------------------
constexpr int kLaneWO = 2, kLaneNB = 2, kLaneWB = 2, kLaneJ = 4;

// lane src's value of v (every lane of the wavefront takes part)
__device__ __forceinline__ double2 lane_read(double2 v, int src) {
  return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

__global__ __launch_bounds__(64) void rk4_lane_kernel(Rk4Args a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const PackDesc pk = a.packs[blockIdx.x];
  const int n = pk.n, n2 = n * n, E = pk.m * n2;
  const PackLds L = carve(smem, pk);
  const BlobLayout BL = blob_layout(n, pk.wo, pk.nb, pk.wb, pk.nc, pk.wc);
  const int tid = threadIdx.x;

  for (int b = tid; b < pk.m; b += 64) {
    const int id = a.order[pk.first + b];
    L.ids[b] = id;
    L.off[b] = a.inst[id].rho_off;
    if (a.status) a.status[id] = 0;
  }
  stage_blobs(L.blobs, pk, a.order, a.inst, a.ops, 0);
  __syncthreads();

  // this lane's element (i, j) of pack instance b; padding lanes (tid >= E)
  // get zero coefficients and read themselves
  const bool own = tid < E;
  const int b = own ? tid / n2 : 0, r = own ? tid - b * n2 : 0;
  const int i = r / n, j = r - i * n, base = b * n2;
  const int wo = pk.wo, nb = pk.nb, wb = pk.wb, wc = pk.wc, nj = pk.nc * pk.wc * pk.wc;
  const double2 zero = make_double2(0.0, 0.0);
  double2 dsum = zero, ao[kLaneWO], bo[kLaneWO], qd[kLaneNB], qa[kLaneNB][kLaneWB],
          qb[kLaneNB][kLaneWB], jp[kLaneJ];
  int as[kLaneWO], bs[kLaneWO], qas[kLaneNB][kLaneWB], qbs[kLaneNB][kLaneWB], js[kLaneJ];
  double cf[kLaneNB][7];
#pragma unroll
  for (int w = 0; w < kLaneWO; ++w) {
    ao[w] = bo[w] = zero;
    as[w] = bs[w] = tid;
  }
#pragma unroll
  for (int q = 0; q < kLaneNB; ++q) {
    qd[q] = zero;
#pragma unroll
    for (int w = 0; w < kLaneWB; ++w) {
      qa[q][w] = qb[q][w] = zero;
      qas[q][w] = qbs[q][w] = tid;
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) cf[q][k] = 0.0;
  }
#pragma unroll
  for (int t = 0; t < kLaneJ; ++t) {
    jp[t] = zero;
    js[t] = tid;
  }
  if (own) {
    const OpView op = make_view(L.blobs + (size_t)b * pk.blob_stride, BL);
    dsum = cadd(op.D[i], cconj(op.D[j]));
#pragma unroll
    for (int w = 0; w < kLaneWO; ++w)
      if (w < wo) {
        ao[w] = op.Oval[w * n + i];
        as[w] = base + op.Ocol[w * n + i] * n + j;
        bo[w] = op.Oval[w * n + j];
        bs[w] = base + i * n + op.Ocol[w * n + j];
      }
#pragma unroll
    for (int q = 0; q < kLaneNB; ++q)
      if (q < nb) {
        qd[q] = cadd(op.DB[q * n + i], cconj(op.DB[q * n + j]));
        const double2 *OB = op.OBval + q * wb * n;
        const int32_t *OC = op.OBcol + q * wb * n;
#pragma unroll
        for (int w = 0; w < kLaneWB; ++w)
          if (w < wb) {
            qa[q][w] = OB[w * n + i];
            qas[q][w] = base + OC[w * n + i] * n + j;
            qb[q][w] = OB[w * n + j];
            qbs[q][w] = base + i * n + OC[w * n + j];
          }
        if (a.fn) {
          const double *p = a.fn + 7 * ((int64_t)L.ids[b] * a.n_ctrl + q);
#pragma unroll
          for (int k = 0; k < 7; ++k) cf[q][k] = p[k];
        }
      }
    // jump products p = J_k[i][w] conj(J_k[j][v]) with source (c_i, c_j),
    // in the order k, w, v
#pragma unroll
    for (int t = 0; t < kLaneJ; ++t)
      if (t < nj) {
        const int k = t / (wc * wc), w = (t / wc) % wc, v = t % wc;
        const double2 *Jv = op.Jval + k * wc * n;
        const int32_t *Jc = op.Jcol + k * wc * n;
        jp[t] = cmul(Jv[w * n + i], cconj(Jv[v * n + j]));
        js[t] = base + Jc[w * n + i] * n + Jc[v * n + j];
      }
  }
  double2 rho = own ? reinterpret_cast<const double2 *>(a.rho0)[L.off[b] + r] : zero;

  const bool want_expect = a.expect != nullptr && a.n_e > 0;
  int next_out = 0;
  const double h = a.h;
  for (int st = 0;; ++st) {
    // outputs due after st steps (st = 0: the initial state)
    while (next_out < a.n_t && a.out_step[next_out] == st) {
      __syncthreads();
      if (own) {
        L.Y[tid] = rho;
        if (a.states)
          reinterpret_cast<double2 *>(a.states)[(int64_t)next_out * a.state_elems + L.off[b] + r] =
              rho;
      }
      __syncthreads();
      if (want_expect) write_outputs<64>(a, pk, L, next_out);
      ++next_out;
    }
    if (st == a.nsteps) break;

    // amplitudes: a piecewise-constant segment value for the whole step, or
    // the closed form at each stage's time (those of rk4_stage_controls())
    double u[kLaneNB];
    const int seg = a.seg_of_step[st];
#pragma unroll
    for (int q = 0; q < kLaneNB; ++q)
      u[q] = (own && q < nb && !a.fn && seg >= 0)
                 ? a.u[((int64_t)L.ids[b] * a.n_ctrl + q) * a.n_seg + seg] : 0.0;
    double2 yn = rho, acc = zero;
    for (int stage = 0; stage < 4; ++stage) {
      const double cnext = stage < 2 ? 0.5 * h : (stage == 2 ? h : 0.0);
      const double wgt = (stage == 0 || stage == 3) ? 1.0 : 2.0;
      if (a.fn) {
        const double tb = a.t0 + (double)st * a.h;
        const double ts = stage == 0 ? tb : (stage == 3 ? tb + a.h : tb + 0.5 * a.h);
#pragma unroll
        for (int q = 0; q < kLaneNB; ++q) u[q] = q < nb ? coeff_fn_at(cf[q], ts) : 0.0;
      }
      // the sources, read from their lanes before any product
      double2 ya[kLaneWO], yb[kLaneWO], yqa[kLaneNB][kLaneWB], yqb[kLaneNB][kLaneWB], yj[kLaneJ];
#pragma unroll
      for (int w = 0; w < kLaneWO; ++w)
        if (w < wo) {
          ya[w] = lane_read(yn, as[w]);
          yb[w] = lane_read(yn, bs[w]);
        }
#pragma unroll
      for (int q = 0; q < kLaneNB; ++q)
#pragma unroll
        for (int w = 0; w < kLaneWB; ++w)
          if (q < nb && w < wb) {
            yqa[q][w] = lane_read(yn, qas[q][w]);
            yqb[q][w] = lane_read(yn, qbs[q][w]);
          }
#pragma unroll
      for (int t = 0; t < kLaneJ; ++t)
        if (t < nj) yj[t] = lane_read(yn, js[t]);
      // (L y)_ij in the order of lindblad_elem()
      double2 kv = cmul(dsum, yn);
#pragma unroll
      for (int w = 0; w < kLaneWO; ++w)
        if (w < wo) kv = cfma(ao[w], ya[w], kv);
#pragma unroll
      for (int w = 0; w < kLaneWO; ++w)
        if (w < wo) kv = cfma_conj(bo[w], yb[w], kv);
#pragma unroll
      for (int q = 0; q < kLaneNB; ++q)
        if (q < nb && u[q] != 0.0) {
          double2 tq = cmul(qd[q], yn);
#pragma unroll
          for (int w = 0; w < kLaneWB; ++w)
            if (w < wb) tq = cfma(qa[q][w], yqa[q][w], tq);
#pragma unroll
          for (int w = 0; w < kLaneWB; ++w)
            if (w < wb) tq = cfma_conj(qb[q][w], yqb[q][w], tq);
          kv = caxpy(u[q], tq, kv);
        }
#pragma unroll
      for (int t = 0; t < kLaneJ; ++t)
        if (t < nj) kv = cfma(jp[t], yj[t], kv);
      acc = caxpy(wgt, kv, acc);
      yn = caxpy(cnext, kv, rho);
    }
    rho = caxpy(h / 6.0, acc, rho);
  }

  if (a.rho_out && own) reinterpret_cast<double2 *>(a.rho_out)[L.off[b] + r] = rho;
  if (a.counts)
    for (int bb = tid; bb < pk.m; bb += 64) {
      a.counts[2 * (int64_t)L.ids[bb]] = a.nsteps;
      a.counts[2 * (int64_t)L.ids[bb] + 1] = 0;
    }
}

// ---------------------------------------------------------------------------
// Resident fixed-step RK4, column-owner layout.  The pack's m instances form
// C = m*n columns; thread t < C*G owns column c = t mod C (instance b, column
// j) and rows i = g, g+G, g+2G, ... with g = t div C.
//   * Column-j operator data (conj of D_j, of the off-diagonal entries of row
//     j of A, of the jump coefficients of row j, and their column indices)
//     are loaded into registers once.
//   * Row-i column indices (off-diagonal of A, jump sources) of each owned
//     row are packed 8 bits apiece into one register, so the y gathers never
//     wait on an index load; row-i values are LDS reads that all lanes of a
//     wave share (broadcasts).
//   * Rows past n are computed on row n-1 and discarded (no branches).
// The operator shape (off-diagonal width WO, number of monomial collapse
// operators NC, number of control terms NB with width kColWB) is a template
// parameter.  Element arithmetic is in the same order as lindblad_elem(), so
// both layouts give identical bits.
// ---------------------------------------------------------------------------
template <int WO, int NC, int NB>
struct ColData {
  double2 dj;
  int ocol[WO > 0 ? WO : 1];
  double2 oval[WO > 0 ? WO : 1];     // conj(O_jw)
  int jcol[NC > 0 ? NC : 1];
  double2 jval[NC > 0 ? NC : 1];     // conj(J_kj)
  double2 dbj[NB > 0 ? NB : 1];
  int obcol[NB > 0 ? NB : 1][kColWB];
  double2 obval[NB > 0 ? NB : 1][kColWB];
};

template <int WO, int NC, int NB>
__device__ __forceinline__ void load_column(ColData<WO, NC, NB> &cd, const OpView &op, int j) {
  const int n = op.n;
  cd.dj = cconj(op.D[j]);
#pragma unroll
  for (int w = 0; w < WO; ++w) {
    cd.ocol[w] = op.Ocol[w * n + j];
    cd.oval[w] = cconj(op.Oval[w * n + j]);
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    cd.jcol[k] = op.Jcol[k * n + j];
    cd.jval[k] = cconj(op.Jval[k * n + j]);
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    cd.dbj[q] = cconj(op.DB[q * n + j]);
#pragma unroll
    for (int w = 0; w < kColWB; ++w) {
      const bool on = w < op.wb;
      cd.obcol[q][w] = on ? op.OBcol[(q * op.wb + w) * n + j] : j;
      cd.obval[q][w] = on ? cconj(op.OBval[(q * op.wb + w) * n + j]) : make_double2(0.0, 0.0);
    }
  }
}

// Row-i column indices, 8 bits each: WO off-diagonal columns of A, then the
// NC jump sources.
template <int WO, int NC>
__device__ __forceinline__ uint32_t row_indices(const OpView &op, int i) {
  const int n = op.n;
  uint32_t v = 0;
#pragma unroll
  for (int w = 0; w < WO; ++w) v |= (uint32_t)op.Ocol[w * n + i] << (8 * w);
#pragma unroll
  for (int k = 0; k < NC; ++k) v |= (uint32_t)op.Jcol[k * n + i] << (8 * (WO + k));
  return v;
}

__device__ __forceinline__ int field8(uint32_t v, int f) { return (int)((v >> (8 * f)) & 255u); }
// 24-bit multiply: full rate on CDNA (a 32-bit multiply is quarter rate);
// every product here is below 2^24.
__device__ __forceinline__ int mul24(int a, int b) { return (int)__umul24((unsigned)a, (unsigned)b); }

// Control term q of the column layout, (B_q y + y B_q^+)_ij with the column-j
// data in registers: the arithmetic of two_sided() in its order (exactly-zero
// parts skipped under RE).  Yrow = Y + i n.
template <int WO, int NC, int NB, bool RE>
__device__ __forceinline__ double2 control_col(const OpView &op, const ColData<WO, NC, NB> &cd,
                                               const double2 *Y, const double2 *Yrow, int i,
                                               int j, double2 yij, int q) {
  const int n = op.n, wb = op.wb;
  const double2 *OB = op.OBval + q * wb * n;
  const int32_t *OC = op.OBcol + q * wb * n;
  double2 t = cmul(cadd(op.DB[q * n + i], cd.dbj[q]), yij);
#pragma unroll
  for (int w = 0; w < kColWB; ++w)
    if (w < wb) {
      const double2 yv = Y[mul24(OC[w * n + i], n) + j];
      if (RE) {
        const double o = reinterpret_cast<const double *>(OB + w * n + i)[1];
        t = make_double2(fma(-o, yv.y, t.x), fma(o, yv.x, t.y));
      } else {
        t = cfma(OB[w * n + i], yv, t);
      }
    }
#pragma unroll
  for (int w = 0; w < kColWB; ++w)
    if (w < wb) {
      const double2 yv = Yrow[cd.obcol[q][w]];
      if (RE)
        t = make_double2(fma(-cd.obval[q][w].y, yv.y, t.x), fma(cd.obval[q][w].y, yv.x, t.y));
      else
        t = cfma(cd.obval[q][w], yv, t);
    }
  return t;
}

// (L y)_ij with the column-j data in registers; same operation order as
// lindblad_elem().  RE: the off-diagonal entries of A (and of the control
// terms) are purely imaginary and the jump coefficients real, which holds for
// a real Hamiltonian with collapse operators whose C^+C are diagonal; the
// vanishing parts are skipped, which changes no bit of the result (they only
// ever add exact zeros).
template <int WO, int NC, int NB, bool RE>
__device__ __forceinline__ double2 lindblad_col(const OpView &op, const ColData<WO, NC, NB> &cd,
                                                const double2 *Y, int i, uint32_t ri, int j,
                                                double2 yij, const double *uq) {
  const int n = op.n;
  const double2 *Yrow = Y + mul24(i, n);
  double2 acc = cmul(cadd(op.D[i], cd.dj), yij);
#pragma unroll
  for (int w = 0; w < WO; ++w) {
    const double2 yv = Y[mul24(field8(ri, w), n) + j];
    if (RE) {
      const double o = reinterpret_cast<const double *>(op.Oval + w * n + i)[1];
      acc = make_double2(fma(-o, yv.y, acc.x), fma(o, yv.x, acc.y));
    } else {
      acc = cfma(op.Oval[w * n + i], yv, acc);
    }
  }
#pragma unroll
  for (int w = 0; w < WO; ++w) {
    const double2 yv = Yrow[cd.ocol[w]];
    if (RE)
      acc = make_double2(fma(-cd.oval[w].y, yv.y, acc.x), fma(cd.oval[w].y, yv.x, acc.y));
    else
      acc = cfma(cd.oval[w], yv, acc);
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const double u = uq[q];
    if (u != 0.0) acc = caxpy(u, control_col<WO, NC, NB, RE>(op, cd, Y, Yrow, i, j, yij, q), acc);
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const double2 yv = Y[mul24(field8(ri, WO + k), n) + cd.jcol[k]];
    if (RE) {
      const double p = reinterpret_cast<const double *>(op.Jval + k * n + i)[0] * cd.jval[k].x;
      acc = make_double2(fma(p, yv.x, acc.x), fma(p, yv.y, acc.y));
    } else {
      const double2 p = cmul(op.Jval[k * n + i], cd.jval[k]);
      acc = cfma(p, yv, acc);
    }
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Row records (column-owner kernels).  One record per row i of an instance,
// built in LDS from the op blob: the byte offsets, relative to the
// instance's stage input, of the rows the row-i products read (own row
// i*n*16, off-diagonal sources Ocol[w][i]*n*16, jump sources
// Jcol[k][i]*n*16, control sources OBcol[q][w][i]*n*16), then the row's
// coefficients D_i, Oval[w][i], Jval[k][i], DB[q][i], OBval[q][w][i].  With
// the column-j positions in registers, each y gather is one add on a record
// field and each coefficient an immediate offset from the record address.
// Records are an odd number of 16-byte units, so lanes reading consecutive
// rows hit distinct LDS banks.
// ---------------------------------------------------------------------------
template <int WO, int NC, int NB>
struct Rec {
  static constexpr int NH = 1 + WO + NC + NB * kColWB;   // header ints
  static constexpr int H = rec_hdr_bytes(WO, NC, NB);
  static constexpr int S = rec_bytes(WO, NC, NB);
  // coefficient slots (double2) after the header
  static constexpr int D = 0, O = 1, J = 1 + WO, CB = 1 + WO + NC, CQ = 1 + kColWB;
};

template <int WO, int NC, int NB>
__device__ void stage_records(uint8_t *dst, const PackDesc &pk, const int32_t *order,
                              const InstDesc *inst, const uint8_t *pool, int adjoint) {
  using RL = Rec<WO, NC, NB>;
  const int n = pk.n, n16 = 16 * n;
  const BlobLayout BL = blob_layout(n, pk.wo, pk.nb, pk.wb, pk.nc, pk.wc);
  for (int idx = threadIdx.x; idx < pk.m * n; idx += blockDim.x) {
    const int b = idx / n, i = idx - b * n;
    const InstDesc &d = inst[order[pk.first + b]];
    const OpView op = make_view(pool + (adjoint ? d.adj_off : d.ops_off), BL);
    uint8_t *r = dst + (size_t)b * pk.blob_stride + i * RL::S;
    int32_t *hd = reinterpret_cast<int32_t *>(r);
    double2 *v = reinterpret_cast<double2 *>(r + RL::H);
    hd[0] = i * n16;
    v[RL::D] = op.D[i];
#pragma unroll
    for (int w = 0; w < WO; ++w) {
      hd[1 + w] = op.Ocol[w * n + i] * n16;
      v[RL::O + w] = op.Oval[w * n + i];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      hd[1 + WO + k] = op.Jcol[k * n + i] * n16;
      v[RL::J + k] = op.Jval[k * n + i];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      v[RL::CB + q * RL::CQ] = op.DB[q * n + i];
#pragma unroll
      for (int w = 0; w < kColWB; ++w) {
        const bool on = w < op.wb;
        hd[1 + WO + NC + q * kColWB + w] = (on ? op.OBcol[(q * op.wb + w) * n + i] : i) * n16;
        v[RL::CB + q * RL::CQ + 1 + w] =
            on ? op.OBval[(q * op.wb + w) * n + i] : make_double2(0.0, 0.0);
      }
    }
#pragma unroll
    for (int t = RL::NH; t < RL::H / 4; ++t) hd[t] = 0;
  }
}

// Column-j data in registers: conjugated coefficients of row j and the LDS
// byte addresses of the column-j entries the products read (row 0; a record
// offset selects the row).
template <int WO, int NC, int NB>
struct ColPos {
  double2 dj;
  double2 oval[WO > 0 ? WO : 1];     // conj(O_jw)
  double2 jval[NC > 0 ? NC : 1];     // conj(J_kj)
  double2 dbj[NB > 0 ? NB : 1];
  double2 obval[NB > 0 ? NB : 1][kColWB];
  uint32_t ybj;                      // Y_b[0][j]
  uint32_t yo[WO > 0 ? WO : 1];      // Y_b[0][Ocol[w][j]]
  uint32_t yj[NC > 0 ? NC : 1];      // Y_b[0][Jcol[k][j]]
  uint32_t yob[NB > 0 ? NB : 1][kColWB];
};

template <int WO, int NC, int NB>
__device__ __forceinline__ void load_column_pos(ColPos<WO, NC, NB> &cd, const OpView &op, int j,
                                                uint32_t yb) {
  const int n = op.n;
  cd.dj = cconj(op.D[j]);
  cd.ybj = yb + 16 * j;
#pragma unroll
  for (int w = 0; w < WO; ++w) {
    cd.yo[w] = yb + 16 * op.Ocol[w * n + j];
    cd.oval[w] = cconj(op.Oval[w * n + j]);
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    cd.yj[k] = yb + 16 * op.Jcol[k * n + j];
    cd.jval[k] = cconj(op.Jval[k * n + j]);
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    cd.dbj[q] = cconj(op.DB[q * n + j]);
#pragma unroll
    for (int w = 0; w < kColWB; ++w) {
      const bool on = w < op.wb;
      cd.yob[q][w] = yb + 16 * (on ? op.OBcol[(q * op.wb + w) * n + j] : j);
      cd.obval[q][w] = on ? cconj(op.OBval[(q * op.wb + w) * n + j]) : make_double2(0.0, 0.0);
    }
  }
}

// (L y)_ij from the row-i record at LDS byte address rec and the column-j
// registers; the arithmetic of lindblad_col() in the same order.
template <int WO, int NC, int NB, bool RE>
__device__ __forceinline__ double2 lindblad_rec(const uint8_t *base, uint32_t rec,
                                                const ColPos<WO, NC, NB> &cd, double2 yij,
                                                const double *uq, int wb) {
  using RL = Rec<WO, NC, NB>;
  int32_t hd[RL::H / 4];
#pragma unroll
  for (int t = 0; t < RL::H / 16; ++t) {
    const int4 q = *reinterpret_cast<const int4 *>(base + rec + 16 * t);
    hd[4 * t] = q.x;
    hd[4 * t + 1] = q.y;
    hd[4 * t + 2] = q.z;
    hd[4 * t + 3] = q.w;
  }
  const double2 *v = reinterpret_cast<const double2 *>(base + rec + RL::H);
  auto Y = [&](uint32_t addr) { return *reinterpret_cast<const double2 *>(base + addr); };
  double2 acc = cmul(cadd(v[RL::D], cd.dj), yij);
#pragma unroll
  for (int w = 0; w < WO; ++w) {
    const double2 yv = Y(cd.ybj + hd[1 + w]);
    if (RE) {
      const double o = reinterpret_cast<const double *>(v + RL::O + w)[1];
      acc = make_double2(fma(-o, yv.y, acc.x), fma(o, yv.x, acc.y));
    } else {
      acc = cfma(v[RL::O + w], yv, acc);
    }
  }
#pragma unroll
  for (int w = 0; w < WO; ++w) {
    const double2 yv = Y(cd.yo[w] + hd[0]);
    if (RE)
      acc = make_double2(fma(-cd.oval[w].y, yv.y, acc.x), fma(cd.oval[w].y, yv.x, acc.y));
    else
      acc = cfma(cd.oval[w], yv, acc);
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const double u = uq[q];
    if (u != 0.0) {
      const double2 *cv = v + RL::CB + q * RL::CQ;
      double2 t = cmul(cadd(cv[0], cd.dbj[q]), yij);
#pragma unroll
      for (int w = 0; w < kColWB; ++w)
        if (w < wb) {
          const double2 yv = Y(cd.ybj + hd[1 + WO + NC + q * kColWB + w]);
          if (RE) {
            const double o = reinterpret_cast<const double *>(cv + 1 + w)[1];
            t = make_double2(fma(-o, yv.y, t.x), fma(o, yv.x, t.y));
          } else {
            t = cfma(cv[1 + w], yv, t);
          }
        }
#pragma unroll
      for (int w = 0; w < kColWB; ++w)
        if (w < wb) {
          const double2 yv = Y(cd.yob[q][w] + hd[0]);
          if (RE)
            t = make_double2(fma(-cd.obval[q][w].y, yv.y, t.x), fma(cd.obval[q][w].y, yv.x, t.y));
          else
            t = cfma(cd.obval[q][w], yv, t);
        }
      acc = caxpy(u, t, acc);
    }
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const double2 yv = Y(cd.yj[k] + hd[1 + WO + k]);
    if (RE) {
      const double p = reinterpret_cast<const double *>(v + RL::J + k)[0] * cd.jval[k].x;
      acc = make_double2(fma(p, yv.x, acc.x), fma(p, yv.y, acc.y));
    } else {
      const double2 p = cmul(v[RL::J + k], cd.jval[k]);
      acc = cfma(p, yv, acc);
    }
  }
  return acc;
}

// Per-slot constants of the Hermitian kernel for real structure without
// control terms: D_i + conj(D_j), Im O_iw, the jump products
// Re J_ik Re J_jk and the row-i column indices (8 bits each).  They are the
// only row-i data an element needs, so the element reads nothing from LDS
// but the y gathers.
template <int WO, int NC>
struct SlotC {
  double2 dsum;
  double o[WO > 0 ? WO : 1];
  double p[NC > 0 ? NC : 1];
  uint32_t ri;
};

template <int WO, int NC>
__device__ __forceinline__ void load_slot(SlotC<WO, NC> &s, const OpView &op,
                                          const ColPos<WO, NC, 0> &cd, int i) {
  const int n = op.n;
  s.dsum = cadd(op.D[i], cd.dj);
#pragma unroll
  for (int w = 0; w < WO; ++w) s.o[w] = reinterpret_cast<const double *>(op.Oval + w * n + i)[1];
#pragma unroll
  for (int k = 0; k < NC; ++k)
    s.p[k] = reinterpret_cast<const double *>(op.Jval + k * n + i)[0] * cd.jval[k].x;
  s.ri = row_indices<WO, NC>(op, i);
}

// (L y)_ij from the slot constants; the arithmetic of lindblad_col() (real
// structure, no control terms) in the same order.  rowoff = i*n*16.
template <int WO, int NC>
__device__ __forceinline__ double2 lindblad_slot(const uint8_t *base, const ColPos<WO, NC, 0> &cd,
                                                 const SlotC<WO, NC> &s, uint32_t rowoff,
                                                 int n16, double2 yij) {
  auto Y = [&](uint32_t addr) { return *reinterpret_cast<const double2 *>(base + addr); };
  double2 acc = cmul(s.dsum, yij);
#pragma unroll
  for (int w = 0; w < WO; ++w) {
    const double2 yv = Y(cd.ybj + mul24(field8(s.ri, w), n16));
    acc = make_double2(fma(-s.o[w], yv.y, acc.x), fma(s.o[w], yv.x, acc.y));
  }
#pragma unroll
  for (int w = 0; w < WO; ++w) {
    const double2 yv = Y(cd.yo[w] + rowoff);
    acc = make_double2(fma(-cd.oval[w].y, yv.y, acc.x), fma(cd.oval[w].y, yv.x, acc.y));
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const double2 yv = Y(cd.yj[k] + mul24(field8(s.ri, WO + k), n16));
    acc = make_double2(fma(s.p[k], yv.x, acc.x), fma(s.p[k], yv.y, acc.y));
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Resident fixed-step RK4 for Hermitian rho0 (density matrices).  rho0 = rho0^+
// makes every stage input and every L(y) Hermitian, so each unordered pair
// {i, j} is computed once and its mirror written as the conjugate.  Threads
// are laid out as in the column-owner kernel (thread t < m*n*G owns column j
// of instance b), but column j owns the rows i = (j + d) mod n for
// d = g, g+G, ... <= floor(n/2): every pair exactly once (for even n the pair
// at d = n/2 goes to the smaller column index), n/2 + 1 rows per column, so
// the threads of an instance stay balanced.  The row index then differs from
// lane to lane; for real structure without control terms (the Jaynes-Cummings
// sweep, one off-diagonal and two jump columns per row) each slot keeps its
// row data in registers (SlotC) and an element reads nothing from LDS but its
// y gathers; otherwise the row-i records are read.  The input is read as its Hermitian part; an instance whose rho0 is
// not Hermitian to 1e-12 relative gets status 9 (LME_ENOTHERM).
// ---------------------------------------------------------------------------
template <int T, int EPT, int WO, int NC, int NB, bool RE>
__global__ __launch_bounds__(T) void rk4_herm_kernel(Rk4Args a) {
  using RL = Rec<WO, NC, NB>;
  constexpr bool SLOTS = herm_slots(RE, WO, NC, NB);
  extern __shared__ __align__(16) uint8_t smem[];
  const PackDesc pk = a.packs[blockIdx.x];
  const int n = pk.n, n2 = n * n, C = pk.m * n, G = pk.G, ept = pk.ept;
  const int R = n / 2 + 1;  // row slots per column
  const PackLds L = carve(smem, pk);
  const int tid = threadIdx.x;

  for (int bb = tid; bb < pk.m; bb += T) {
    const int id = a.order[pk.first + bb];
    L.ids[bb] = id;
    L.off[bb] = a.inst[id].rho_off;
    if (a.status) a.status[id] = 0;
  }
  if (!SLOTS) stage_records<WO, NC, NB>(L.blobs, pk, a.order, a.inst, a.ops, 0);
  __syncthreads();

  const bool active = tid < C * G;
  const int g = active ? tid / C : 0;
  const int c = active ? tid - g * C : 0;
  const int b = c / n, j = c - b * n;
  double2 *Yb = L.Y + b * n2;
  const uint32_t yb = (uint32_t)(reinterpret_cast<uint8_t *>(Yb) - smem);
  const uint32_t recb = (uint32_t)(L.blobs + (size_t)b * pk.blob_stride - smem);
  const uint32_t ybjn = yb + 16 * n * j;  // Y_b[j][0]
  const OpView gop = make_view(a.ops + a.inst[L.ids[b]].ops_off,
                               blob_layout(n, pk.wo, pk.nb, pk.wb, pk.nc, pk.wc));
  ColPos<WO, NC, NB> cd;
  load_column_pos<WO, NC, NB>(cd, gop, j, yb);

  // Slot r: row offset d = min(g + r*G, n/2), row i = j + d mod n (past the
  // last offset the slot repeats it: computed, never stored).  pos[r] packs
  // the row's record offset (high half) and 16*i (low half).  The thread
  // owns its slots r < nown.
  int nown = 0;
  if (active) {
    const int Rown = ((n & 1) == 0 && 2 * j >= n) ? R - 1 : R;
    nown = g < Rown ? (Rown - g + G - 1) / G : 0;
  }
  uint32_t pos[EPT];
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    int i = j + min(g + r * G, R - 1);
    i = i >= n ? i - n : i;
    pos[r] = ((uint32_t)(i * RL::S) << 16) | (uint32_t)(16 * i);
  }
  auto row_of = [](uint32_t p) { return (int)((p & 0xffffu) >> 4); };
  SlotC<WO, NC> sc[SLOTS ? EPT : 1];
  if constexpr (SLOTS) {
#pragma unroll
    for (int r = 0; r < EPT; ++r) load_slot<WO, NC>(sc[r], gop, cd, row_of(pos[r]));
  }
  // stage input element (i, j) and its mirror into LDS; the mirror goes
  // first, so on the diagonal the element itself is what remains
  auto put = [&](uint32_t p, double2 v) {
    const uint32_t i16 = p & 0xffffu;
    *reinterpret_cast<double2 *>(smem + ybjn + i16) = cconj(v);
    *reinterpret_cast<double2 *>(smem + cd.ybj + mul24(i16, n)) = v;
  };
  // element (i, j) and its mirror into global memory
  auto put_global = [&](double2 *dst, uint32_t p, double2 v) {
    const int i = row_of(p);
    dst[i * n + j] = v;
    if (i != j) dst[j * n + i] = cconj(v);
  };

  double2 rho[EPT], acc[EPT], yn[EPT];
  const double2 *rho0 = reinterpret_cast<const double2 *>(a.rho0) + L.off[b];
  bool not_herm = false;
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    rho[r] = make_double2(0.0, 0.0);
    if (r < nown) {
      const int i = row_of(pos[r]);
      const double2 x = rho0[i * n + j], y = rho0[j * n + i];
      const double dx = x.x - y.x, dy = x.y + y.y;
      not_herm |= dx * dx + dy * dy > 2e-24 * (x.x * x.x + x.y * x.y + y.x * y.x + y.y * y.y);
      rho[r] = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
    }
  }
  if (not_herm && a.status) a.status[L.ids[b]] = 9;  // LME_ENOTHERM

  const bool want_expect = a.expect != nullptr && a.n_e > 0;
  int next_out = 0;
  const double h = a.h;
  for (int st = 0;; ++st) {
    // an output step leaves rho, the first stage's input, in LDS: without
    // control terms that stage then needs neither its store nor its barriers
    bool staged = false;
    while (next_out < a.n_t && a.out_step[next_out] == st) {
      staged = true;
      __syncthreads();
#pragma unroll
      for (int r = 0; r < EPT; ++r)
        if (r < nown) {
          uint32_t p = pos[r];
          asm volatile("" : "+v"(p));
          put(p, rho[r]);
          if (a.states)
            put_global(reinterpret_cast<double2 *>(a.states) +
                           (int64_t)next_out * a.state_elems + L.off[b], p, rho[r]);
        }
      __syncthreads();
      if (want_expect) write_outputs<T>(a, pk, L, next_out);
      ++next_out;
    }
    if (st == a.nsteps) break;

#pragma unroll
    for (int r = 0; r < EPT; ++r) {
      yn[r] = rho[r];
      acc[r] = make_double2(0.0, 0.0);
    }
    for (int stage = 0; stage < 4; ++stage) {
      const double cnext = stage < 2 ? 0.5 * h : (stage == 2 ? h : 0.0);
      const double wgt = (stage == 0 || stage == 3) ? 1.0 : 2.0;
      if (!(NB == 0 && stage == 0 && staged)) {
        __syncthreads();
        if (NB > 0 && (stage == 0 || a.fn))
          rk4_stage_controls(a, pk, L.ids, L.u, st, stage, tid, T);
#pragma unroll
        for (int r = 0; r < EPT; ++r)
          if (r < nown) {
            uint32_t p = pos[r];
            asm volatile("" : "+v"(p));
            put(p, yn[r]);
          }
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < EPT; ++r) {
        if (r < ept) {
          uint32_t p = pos[r];
          asm volatile("" : "+v"(p));
          double2 kv;
          if constexpr (SLOTS)
            kv = lindblad_slot<WO, NC>(smem, cd, sc[r], mul24(p & 0xffffu, n), 16 * n, yn[r]);
          else
            kv = lindblad_rec<WO, NC, NB, RE>(smem, recb + (p >> 16), cd, yn[r],
                                              L.u + b * pk.nb, pk.wb);
          // the diagonal of L(y) is real for Hermitian y: drop the rounding
          // residue of its imaginary part (slot 0 of row group 0 is d = 0)
          if (r == 0) kv.y = g == 0 ? 0.0 : kv.y;
          acc[r] = caxpy(wgt, kv, acc[r]);
          yn[r] = caxpy(cnext, kv, rho[r]);
        }
        if (r & 1) __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int r = 0; r < EPT; ++r) rho[r] = caxpy(h / 6.0, acc[r], rho[r]);
  }

  if (a.rho_out) {
#pragma unroll
    for (int r = 0; r < EPT; ++r)
      if (r < nown) put_global(reinterpret_cast<double2 *>(a.rho_out) + L.off[b], pos[r], rho[r]);
  }
  if (a.counts)
    for (int bb = tid; bb < pk.m; bb += T) {
      a.counts[2 * (int64_t)L.ids[bb]] = a.nsteps;
      a.counts[2 * (int64_t)L.ids[bb] + 1] = 0;
    }
}

template <int T, int EPT, int WO, int NC, int NB, bool RE>
__global__ __launch_bounds__(T) void rk4_colown_kernel(Rk4Args a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const PackDesc pk = a.packs[blockIdx.x];
  const int n = pk.n, n2 = n * n, C = pk.m * n, G = pk.G, ept = pk.ept;
  const PackLds L = carve(smem, pk);
  const BlobLayout BL = blob_layout(n, pk.wo, pk.nb, pk.wb, pk.nc, pk.wc);
  const int tid = threadIdx.x;

  for (int b = tid; b < pk.m; b += T) {
    const int id = a.order[pk.first + b];
    L.ids[b] = id;
    L.off[b] = a.inst[id].rho_off;
    if (a.status) a.status[id] = 0;
  }
  stage_blobs(L.blobs, pk, a.order, a.inst, a.ops, a.adjoint);
  __syncthreads();

  const bool active = tid < C * G;
  const int g = active ? tid / C : 0;
  const int c = active ? tid - g * C : 0;
  const int b = c / n, j = c - b * n;
  const OpView op = make_view(L.blobs + (size_t)b * pk.blob_stride, BL);
  double2 *Yb = L.Y + b * n2;
  ColData<WO, NC, NB> cd;
  load_column<WO, NC, NB>(cd, op, j);

  // Slot r holds row g + r*G; past n the row is clamped to n-1 (computed,
  // never stored).  Rows are re-derived from an opaque copy of g wherever
  // they are used, so no per-row address lives across stages in a register.
  auto row_of = [&](int gg, int r) { return min(gg + r * G, n - 1); };
  auto owns = [&](int gg, int r) { return active && r < ept && gg + r * G < n; };

  double2 rho[EPT], acc[EPT], yn[EPT];
  uint32_t ridx[EPT];
  const double2 *rho0 = reinterpret_cast<const double2 *>(a.rho0);
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    ridx[r] = row_indices<WO, NC>(op, row_of(g, r));
    rho[r] = owns(g, r) ? rho0[L.off[b] + row_of(g, r) * n + j] : make_double2(0.0, 0.0);
  }

  const bool want_expect = a.expect != nullptr && a.n_e > 0;
  int next_out = 0;
  const double h = a.h;
  for (int st = 0;; ++st) {
    // an output step leaves rho, the first stage's input, in LDS: without
    // control terms that stage then needs neither its store nor its barriers
    bool staged = false;
    while (next_out < a.n_t && a.out_step[next_out] == st) {
      staged = true;
      __syncthreads();
      int gg = g;
      asm volatile("" : "+v"(gg));
#pragma unroll
      for (int r = 0; r < EPT; ++r)
        if (owns(gg, r)) {
          const int i = row_of(gg, r);
          Yb[mul24(i, n) + j] = rho[r];
          if (a.states)
            reinterpret_cast<double2 *>(a.states)[(int64_t)next_out * a.state_elems + L.off[b] +
                                                  i * n + j] = rho[r];
        }
      __syncthreads();
      if (want_expect) write_outputs<T>(a, pk, L, next_out);
      ++next_out;
    }
    if (st == a.nsteps) break;

#pragma unroll
    for (int r = 0; r < EPT; ++r) {
      yn[r] = rho[r];
      acc[r] = make_double2(0.0, 0.0);
    }
    for (int stage = 0; stage < 4; ++stage) {
      const double cnext = stage < 2 ? 0.5 * h : (stage == 2 ? h : 0.0);
      const double wgt = (stage == 0 || stage == 3) ? 1.0 : 2.0;
      int gg = g;
      asm volatile("" : "+v"(gg));
      if (!(NB == 0 && stage == 0 && staged)) {
        __syncthreads();
        if (NB > 0 && (stage == 0 || a.fn))
          rk4_stage_controls(a, pk, L.ids, L.u, st, stage, tid, T);
#pragma unroll
        for (int r = 0; r < EPT; ++r)
          if (owns(gg, r)) Yb[mul24(row_of(gg, r), n) + j] = yn[r];
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < EPT; ++r) {
        if (r < ept) {
          uint32_t ri = ridx[r];
          int i = row_of(gg, r);
          asm volatile("" : "+v"(i), "+v"(ri));
          const double2 kv = lindblad_col<WO, NC, NB, RE>(op, cd, Yb, i, ri, j, yn[r],
                                                      L.u + b * pk.nb);
          acc[r] = caxpy(wgt, kv, acc[r]);
          yn[r] = caxpy(cnext, kv, rho[r]);
        }
        if (r & 1) __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int r = 0; r < EPT; ++r) rho[r] = caxpy(h / 6.0, acc[r], rho[r]);
  }

  if (a.rho_out) {
#pragma unroll
    for (int r = 0; r < EPT; ++r)
      if (owns(g, r))
        reinterpret_cast<double2 *>(a.rho_out)[L.off[b] + row_of(g, r) * n + j] = rho[r];
  }
  if (a.counts)
    for (int bb = tid; bb < pk.m; bb += T) {
      a.counts[2 * (int64_t)L.ids[bb]] = a.nsteps;
      a.counts[2 * (int64_t)L.ids[bb] + 1] = 0;
    }
}

// ---------------------------------------------------------------------------
// Resident Dormand-Prince 5(4) with per-instance step control.
// One workgroup integrates one pack; each instance has its own t, h,
// accept/reject history and position in the list of stop points (output
// times and control edges, which every step lands on exactly).  The stage
// input is shared through LDS; each thread keeps rho, the stage input and the
// fifth-order solution of its elements in VGPRs and the seven stage
// derivatives in a global scratch it alone reads and writes.  Per-instance
// norms are reduced in a fixed order (deterministic).
// ---------------------------------------------------------------------------

// Dormand & Prince (1980): stage matrix, fifth-order weights (= last row,
// first-same-as-last) and the embedded fourth-order weights.
__constant__ double kDpA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
// error weights b_i - bhat_i
__constant__ double kDpE[7] = {35.0 / 384 - 5179.0 / 57600,
                               0.0,
                               500.0 / 1113 - 7571.0 / 16695,
                               125.0 / 192 - 393.0 / 640,
                               -2187.0 / 6784 - (-92097.0 / 339200),
                               11.0 / 84 - 187.0 / 2100,
                               0.0 - 1.0 / 40};


__host__ __device__ inline int32_t dp_ctl_bytes(int32_t m) {
  return align16(m * (int32_t)sizeof(DpCtl));
}

// Sum over each instance's n2 entries of buf (LDS doubles) -> out[b];
// waves take instances round-robin, lanes stride the entries, then a
// butterfly: a fixed order.
template <int T>
__device__ void per_instance_sum(const double *buf, int m, int n2, double *out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int b = wave; b < m; b += T / 64) {
    double v = 0.0;
    for (int e = lane; e < n2; e += 64) v += buf[b * n2 + e];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) out[b] = v;
  }
}

// Expectation values of the instances whose out_due >= 0 (their rho is in Y).
template <int T>
__device__ void dp_outputs(const Dp5Args &a, const PackDesc &pk, const PackLds &L,
                           const DpCtl *ctl) {
  const int n = pk.n, n2 = n * n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int task = wave; task < pk.m * a.n_e; task += T / 64) {
    const int b = task / a.n_e, e = task - b * a.n_e;
    const int k = ctl[b].out_due;
    if (k < 0) continue;
    const int id = L.ids[b];
    const InstDesc &d = a.inst[id];
    const int we = d.we;
    const int32_t *Ec = reinterpret_cast<const int32_t *>(a.eops + d.eops_off);
    const double2 *Ev = reinterpret_cast<const double2 *>(
        a.eops + d.eops_off + eops_val_offset(n, we, a.n_e));
    const double2 *Y = L.Y + b * n2;
    double2 part = make_double2(0.0, 0.0);
    for (int i = lane; i < n; i += 64)
      for (int w = 0; w < we; ++w) {
        const int idx = (e * we + w) * n + i;
        part = cfma(Ev[idx], Y[Ec[idx] * n + i], part);
      }
    part = wave_sum(part);
    if (lane == 0) {
      double *dst = a.expect + 2 * (((int64_t)id * a.n_e + e) * a.n_t + k);
      dst[0] = part.x;
      dst[1] = part.y;
    }
  }
}

// COL: column-owner layout (the packs of the column kernels: thread owns
// column j of instance b and rows g, g+G, ...), elements evaluated by
// lindblad_col() with the column-j operator data in registers; otherwise the
// row layout (thread owns pack elements f = t + s*T), lindblad_elem().  Both
// give the same bits; everything but the element evaluation goes through the
// slot's (instance, row, column).
template <int T, int EPT, int WO, int NC, int NB, bool RE, bool COL>
__global__ __launch_bounds__(T) void dp5_resident_kernel(Dp5Args a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const PackDesc pk = a.packs[blockIdx.x];
  const int n = pk.n, n2 = n * n, E = pk.m * n2, m = pk.m;
  const PackLds L = carve(smem, pk);
  DpCtl *ctl = reinterpret_cast<DpCtl *>(smem + pack_lds_bytes(n, m, pk.blob_bytes, pk.nb));
  double *red = reinterpret_cast<double *>(L.Y);   // reduction scratch aliases Y
  double *sums = reinterpret_cast<double *>(L.u);  // (reused only when nb == 0: see below)
  const BlobLayout BL = blob_layout(n, pk.wo, pk.nb, pk.wb, pk.nc, pk.wc);
  const int tid = threadIdx.x;
  double2 *K = reinterpret_cast<double2 *>(a.kbuf);
  const int64_t SE = a.state_elems;
  (void)sums;

  for (int b = tid; b < m; b += T) {
    const int id = a.order[pk.first + b];
    L.ids[b] = id;
    L.off[b] = a.inst[id].rho_off;
    if (a.status) a.status[id] = 0;
    DpCtl c;
    c.t = a.t0;
    c.h = a.h0;
    c.h_try = 0.0;
    c.hs = 0.0;
    c.n_acc = c.n_rej = 0;
    c.stop = 0;
    c.status = 0;
    c.active = a.n_stops > 0;
    c.accept = c.landing = 0;
    c.seg = -1;
    c.k1_seg = -2;
    c.prev_rej = 0;
    c.out_due = 0;   // the initial state is output 0
    c.need_k1 = 1;
    ctl[b] = c;
  }
  stage_blobs(L.blobs, pk, a.order, a.inst, a.ops, 0);
  __syncthreads();

  // yn: the current stage input; after the seventh stage it is the
  // fifth-order solution (the last stage is evaluated at it)
  double2 rho[EPT], yn[EPT];
  uint32_t bij[EPT];
  uint32_t vmask = 0;  // slots this thread owns
  const double2 *rho0 = reinterpret_cast<const double2 *>(a.rho0);
  // column layout: this thread's column and its operator data
  const int C = COL ? m * n : 0, G = COL ? pk.G : 1;
  const bool cactive = COL && tid < C * G;
  const int cg = cactive ? tid / C : 0, cc = cactive ? tid - cg * C : 0;
  const int cb = cc / (COL ? n : 1), cj = cc - cb * n;
  ColData<WO, NC, NB> cd;
  uint32_t ridx[COL ? EPT : 1];
  if constexpr (COL) load_column<WO, NC, NB>(cd, make_view(L.blobs + (size_t)cb * pk.blob_stride, BL), cj);
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    rho[s] = make_double2(0.0, 0.0);
    bij[s] = 0;
    if constexpr (COL) {
      const int i = cg + s * G;
      const OpView op = make_view(L.blobs + (size_t)cb * pk.blob_stride, BL);
      ridx[s] = row_indices<WO, NC>(op, min(i, n - 1));
      bij[s] = pack_bij(cb, min(i, n - 1), cj);
      if (cactive && s < pk.ept && i < n) {
        vmask |= 1u << s;
        rho[s] = rho0[L.off[cb] + i * n + cj];
      }
    } else {
      const int f = tid + s * T;
      if (f < E) {
        vmask |= 1u << s;
        const int b = f / n2, r = f - b * n2;
        const int i = r / n;
        bij[s] = pack_bij(b, i, r - i * n);
        rho[s] = rho0[L.off[b] + r];
      }
    }
  }
  auto valid = [&](int s) { return ((vmask >> s) & 1u) != 0; };
  // pack element index of slot s
  auto flat = [&](int s) {
    if constexpr (COL) return slot_b(bij[s]) * n2 + slot_i(bij[s]) * n + slot_j(bij[s]);
    else return tid + s * T;
  };
  auto goff = [&](uint32_t v) { return L.off[slot_b(v)] + slot_i(v) * n + slot_j(v); };
  auto set_controls = [&](int b, int seg) {
    for (int q = 0; q < pk.nb; ++q)
      L.u[b * pk.nb + q] =
          seg >= 0 ? a.u[((int64_t)L.ids[b] * a.n_ctrl + q) * a.n_seg + seg] : 0.0;
  };
  // writes rho of every instance with a due output to Y, then the outputs
  auto outputs = [&]() {
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      if (valid(s)) {
        const int f = flat(s);
        const int b = slot_b(bij[s]);
        const int k = ctl[b].out_due;
        if (k >= 0) {
          L.Y[f] = rho[s];
          if (a.states)
            reinterpret_cast<double2 *>(a.states)[(int64_t)k * SE + goff(bij[s])] = rho[s];
        }
      }
    }
    __syncthreads();
    if (a.expect && a.n_e > 0) dp_outputs<T>(a, pk, L, ctl);
    __syncthreads();
    for (int b = tid; b < m; b += T) ctl[b].out_due = -1;
    __syncthreads();
  };
  auto elem = [&](int s, const double2 &y) {
    uint32_t v = bij[s];
    asm volatile("" : "+v"(v));  // no per-slot addresses hoisted across steps
    const int b = slot_b(v);
    const OpView op = make_view(L.blobs + (size_t)b * pk.blob_stride, BL);
    if constexpr (COL) {
      uint32_t ri = ridx[s];
      asm volatile("" : "+v"(ri));
      return lindblad_col<WO, NC, NB, RE>(op, cd, L.Y + b * n2, slot_i(v), ri, slot_j(v), y,
                                          L.u + b * pk.nb);
    } else {
      return lindblad_elem(op, L.Y + b * n2, slot_i(v), slot_j(v), y, L.u + b * pk.nb);
    }
  };

  outputs();
  if (a.n_stops == 0) goto finish;

  // Starting step (Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4) in
  // the scaled RMS norm, exponent 1/5, with the controls of the first interval.
  if (a.h0 <= 0.0) {
    for (int b = tid; b < m; b += T) set_controls(b, a.n_seg > 0 ? a.stop_seg[0] : -1);
#pragma unroll
    for (int s = 0; s < EPT; ++s)
      if (valid(s)) L.Y[flat(s)] = rho[s];
    __syncthreads();
    double2 f0[EPT];
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      f0[s] = make_double2(0.0, 0.0);
      if (valid(s)) {
        f0[s] = elem(s, rho[s]);
        K[goff(bij[s])] = f0[s];
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      if (valid(s)) {
        const int f = flat(s);
        const double sc = a.atol + a.rtol * hypot(rho[s].x, rho[s].y);
        const double r0 = hypot(rho[s].x, rho[s].y) / sc, r1 = hypot(f0[s].x, f0[s].y) / sc;
        red[f] = r0 * r0;
        red[E + f] = r1 * r1;
      }
    }
    __syncthreads();
    double *d01 = reinterpret_cast<double *>(ctl + m);  // 2m doubles after ctl
    per_instance_sum<T>(red, m, n2, d01);
    per_instance_sum<T>(red + E, m, n2, d01 + m);
    __syncthreads();
    for (int b = tid; b < m; b += T) {
      const double d0 = sqrt(d01[b] / n2), d1 = sqrt(d01[m + b] / n2);
      ctl[b].hs = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
      ctl[b].t = d1;  // keep d1 until h is set
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < EPT; ++s)
      if (valid(s)) {
        const double hs = ctl[slot_b(bij[s])].hs;
        L.Y[flat(s)] = caxpy(hs, f0[s], rho[s]);
      }
    __syncthreads();
    double2 (&f1)[EPT] = yn;
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      f1[s] = make_double2(0.0, 0.0);
      if (valid(s)) f1[s] = elem(s, L.Y[flat(s)]);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      if (valid(s)) {
        const int f = flat(s);
        const double sc = a.atol + a.rtol * hypot(rho[s].x, rho[s].y);
        const double r2 = hypot(f1[s].x - f0[s].x, f1[s].y - f0[s].y) / sc;
        red[f] = r2 * r2;
      }
    }
    __syncthreads();
    per_instance_sum<T>(red, m, n2, d01);
    __syncthreads();
    for (int b = tid; b < m; b += T) {
      DpCtl &c = ctl[b];
      const double hs = c.hs, d1 = c.t;
      const double d2 = sqrt(d01[b] / n2) / hs;
      const double dm = fmax(d1, d2);
      const double h1 = (dm <= 1e-15) ? fmax(1e-6, hs * 1e-3) : pow(0.01 / dm, 0.2);
      c.h = fmin(100.0 * hs, h1);
      c.t = a.t0;
      c.k1_seg = a.n_seg > 0 ? a.stop_seg[0] : -1;   // f0 is the first step's k1
    }
    __syncthreads();
  }

  for (;;) {
    __syncthreads();  // the previous step's decision has been applied everywhere
    // ---- step set-up, one thread per instance
    int any = 0;
    for (int b = tid; b < m; b += T) {
      DpCtl &c = ctl[b];
      if (c.active) {
        if (c.n_acc + c.n_rej >= a.max_steps) {
          c.status = 3;  // LME_EMAXSTEPS
          c.active = 0;
        } else if (c.h < a.h_min) {
          c.status = 4;  // LME_ESTEPUNDERFLOW
          c.active = 0;
        } else {
          const double ts = a.stops[c.stop];
          c.landing = c.h >= ts - c.t;
          c.h_try = c.landing ? ts - c.t : c.h;
          c.seg = a.n_seg > 0 ? a.stop_seg[c.stop] : -1;
          c.need_k1 = c.k1_seg != c.seg;
          set_controls(b, c.seg);
        }
      }
      any |= c.active;
    }
    if (!__syncthreads_or(any)) break;

    // ---- seven stages.  In the column layout every slot of a thread belongs
    // to instance cb, whose step control the stages only read: it is read
    // once per step instead of once per slot and stage.
    int c_active = 0, c_need_k1 = 0;
    double c_h_try = 0.0;
    if constexpr (COL) {
      const DpCtl &c = ctl[cb];
      c_active = c.active;
      c_need_k1 = c.need_k1;
      c_h_try = c.h_try;
    }
    auto ctl_of = [&](int s, int &act, int &nk1, double &ht) {
      if constexpr (COL) {
        act = c_active;
        nk1 = c_need_k1;
        ht = c_h_try;
      } else {
        const DpCtl &c = ctl[slot_b(bij[s])];
        act = c.active;
        nk1 = c.need_k1;
        ht = c.h_try;
      }
    };
    for (int st = 0; st < 7; ++st) {
#pragma unroll
      for (int s = 0; s < EPT; ++s) {
        if (valid(s)) {
          const int f = flat(s);
          int act, nk1;
          double ht;
          ctl_of(s, act, nk1, ht);
          if (act) {
            double2 y = rho[s];
            if (st > 0) {
              const int64_t g = goff(bij[s]);
              double2 acc = make_double2(0.0, 0.0);
              for (int jj = 0; jj < st; ++jj) acc = caxpy(kDpA[st][jj], K[jj * SE + g], acc);
              y = caxpy(ht, acc, y);
            }
            yn[s] = y;
            L.Y[f] = y;
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < EPT; ++s) {
        if (valid(s)) {
          int act, nk1;
          double ht;
          ctl_of(s, act, nk1, ht);
          if (act && (st > 0 || nk1)) K[st * SE + goff(bij[s])] = elem(s, yn[s]);
        }
      }
      __syncthreads();
    }

    // ---- error norm: RMS over the n^2 moduli of e / (atol + rtol max(|rho|, |y5|))
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      if (valid(s)) {
        const int f = flat(s);
        int act, nk1;
        double ht;
        ctl_of(s, act, nk1, ht);
        double v = 0.0;
        if (act) {
          const int64_t g = goff(bij[s]);
          double2 e = make_double2(0.0, 0.0);
          for (int jj = 0; jj < 7; ++jj) e = caxpy(kDpE[jj], K[jj * SE + g], e);
          e = make_double2(ht * e.x, ht * e.y);
          const double sc =
              a.atol + a.rtol * fmax(hypot(rho[s].x, rho[s].y), hypot(yn[s].x, yn[s].y));
          const double r = hypot(e.x, e.y) / sc;
          v = r * r;
        }
        red[f] = v;
      }
    }
    __syncthreads();
    double *errs = reinterpret_cast<double *>(ctl + m);
    per_instance_sum<T>(red, m, n2, errs);
    __syncthreads();
    int due = 0;
    for (int b = tid; b < m; b += T) {
      DpCtl &c = ctl[b];
      c.accept = 0;
      if (!c.active) continue;
      const double err = sqrt(errs[b] / n2);
      c.k1_seg = c.seg;  // k1 now holds f(rho) for this segment
      if (!isfinite(err)) {
        c.status = 5;  // LME_ENONFINITE
        c.active = 0;
      } else if (err <= 1.0) {
        c.accept = 1;
        ++c.n_acc;
        double fac = (err == 0.0) ? 10.0 : 0.9 * pow(err, -0.2);
        fac = fmin(10.0, fmax(0.2, fac));
        if (c.prev_rej && fac > 1.0) fac = 1.0;
        c.prev_rej = 0;
        c.h = c.h_try * fac;
        if (c.landing) {
          c.t = a.stops[c.stop];
          c.out_due = a.stop_out[c.stop];
          due |= c.out_due >= 0;
          if (++c.stop == a.n_stops) c.active = 0;
        } else {
          c.t += c.h_try;
        }
      } else {
        ++c.n_rej;
        c.prev_rej = 1;
        c.h = c.h_try * fmax(0.2, 0.9 * pow(err, -0.2));
      }
    }
    due = __syncthreads_or(due);
    // ---- accepted instances move to the fifth-order solution; k7 -> k1
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      if (valid(s) && ctl[slot_b(bij[s])].accept) {
        rho[s] = yn[s];
        const int64_t g = goff(bij[s]);
        K[g] = K[6 * SE + g];
      }
    }
    if (due) outputs();
  }

finish:
  __syncthreads();
  if (a.rho_out) {
#pragma unroll
    for (int s = 0; s < EPT; ++s)
      if (valid(s)) reinterpret_cast<double2 *>(a.rho_out)[goff(bij[s])] = rho[s];
  }
  for (int b = tid; b < m; b += T) {
    const int id = L.ids[b];
    if (a.counts) {
      a.counts[2 * (int64_t)id] = ctl[b].n_acc;
      a.counts[2 * (int64_t)id + 1] = ctl[b].n_rej;
    }
    if (a.status) a.status[id] = ctl[b].status;
  }
}

// ---------------------------------------------------------------------------
// Cost J = Re Tr(O rho(t1)) under fixed-step RK4 and its gradient with
// respect to the piecewise-constant amplitudes, by the discrete adjoint of
// the RK4 map.  One workgroup per pack: forward pass with a checkpoint every
// ckpt_every steps; backward pass over the checkpoint intervals in reverse,
// each first recomputing its stage inputs Y_1..Y_4 into global scratch, then
// stepping back with
//   kappa_4 = h/6 lambda,              w_4 = L^+ kappa_4,
//   kappa_3 = h/3 lambda + h   w_4,    w_3 = L^+ kappa_3,
//   kappa_2 = h/3 lambda + h/2 w_3,    w_2 = L^+ kappa_2,
//   kappa_1 = h/6 lambda + h/2 w_2,    w_1 = L^+ kappa_1,
//   lambda <- lambda + w_1 + w_2 + w_3 + w_4,
//   dJ/du_q[seg] += sum_i Re <kappa_i, -i[H_q, Y_i]>,
// starting from lambda = O^+ (the gradient of Re Tr(O rho) under the real
// inner product Re Tr(X^+ Y)).  -i[H_q, Y] is the two-sided control term
// B_q Y + Y B_q^+ of the forward operator blob.  The blobs of a pack hold the
// forward operators followed by the adjoint ones.
// COL: the column-owner layout of the column kernels (thread owns column j of
// instance b and rows g, g+G, ...; real structure, monomial jumps, the
// operator shape WO, NC, NQ a template parameter): the column-j data of the
// forward and of the adjoint operator in registers, elements by
// lindblad_col() and control_col(), which give the bits of the row layout.
// ---------------------------------------------------------------------------
template <int T, int EPT, int NQ, int WO = 0, int NC = 0, bool COL = false>
__global__ __launch_bounds__(T) void grad_resident_kernel(GradArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const PackDesc pk = a.packs[blockIdx.x];
  const int n = pk.n, n2 = n * n, E = pk.m * n2, m = pk.m;
  const PackLds L = carve(smem, pk);
  double *sums = reinterpret_cast<double *>(smem + pack_lds_bytes(n, m, pk.blob_bytes, pk.nb));
  double *red = reinterpret_cast<double *>(L.Y);
  const BlobLayout BF = blob_layout(n, pk.wo, pk.nb, pk.wb, pk.nc, pk.wc);
  const BlobLayout BA = blob_layout(n, pk.awo, pk.nb, pk.awb, pk.nc, pk.awc);
  const int tid = threadIdx.x;
  const int64_t SE = a.state_elems;
  const double h = a.h;

  {  // forward blob then adjoint blob of every instance
    const int nv = pk.blob_bytes / 16, nf = pk.fwd_bytes / 16;
    for (int idx = tid; idx < m * nv; idx += T) {
      const int b = idx / nv, r = idx - b * nv;
      const InstDesc &d = a.inst[a.order[pk.first + b]];
      const uint4 *src = r < nf ? reinterpret_cast<const uint4 *>(a.ops + d.ops_off) + r
                                : reinterpret_cast<const uint4 *>(a.adj + d.adj_off) + (r - nf);
      reinterpret_cast<uint4 *>(L.blobs + (size_t)b * pk.blob_stride)[r] = *src;
    }
  }
  for (int b = tid; b < m; b += T) {
    const int id = a.order[pk.first + b];
    L.ids[b] = id;
    L.off[b] = a.inst[id].rho_off;
    for (int q = 0; q < a.n_ctrl * a.n_seg; ++q) a.grad[(int64_t)id * a.n_ctrl * a.n_seg + q] = 0.0;
  }
  __syncthreads();

  double2 rho[EPT], acc[EPT], yn[EPT];
  uint32_t bij[EPT];
  uint32_t vmask = 0;  // slots this thread owns
  // column layout: this thread's column, its operator data and row indices
  const int C = COL ? m * n : 0, G = COL ? pk.G : 1;
  const bool cactive = COL && tid < C * G;
  const int cg = cactive ? tid / C : 0, cc = cactive ? tid - cg * C : 0;
  const int cb = cc / (COL ? n : 1), cj = cc - cb * n;
  ColData<WO, NC, NQ> cdf, cda;
  uint32_t rif[COL ? EPT : 1], ria[COL ? EPT : 1];
  if constexpr (COL) {
    const uint8_t *blob = L.blobs + (size_t)cb * pk.blob_stride;
    load_column<WO, NC, NQ>(cdf, make_view(blob, BF), cj);
    load_column<WO, NC, NQ>(cda, make_view(blob + pk.fwd_bytes, BA), cj);
  }
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    rho[s] = make_double2(0.0, 0.0);
    bij[s] = 0;
    if constexpr (COL) {
      const int i = cg + s * G, ic = min(i, n - 1);
      const uint8_t *blob = L.blobs + (size_t)cb * pk.blob_stride;
      rif[s] = row_indices<WO, NC>(make_view(blob, BF), ic);
      ria[s] = row_indices<WO, NC>(make_view(blob + pk.fwd_bytes, BA), ic);
      bij[s] = pack_bij(cb, ic, cj);
      if (cactive && s < pk.ept && i < n) {
        vmask |= 1u << s;
        rho[s] = reinterpret_cast<const double2 *>(a.rho0)[L.off[cb] + i * n + cj];
      }
    } else {
      const int f = tid + s * T;
      if (f < E) {
        vmask |= 1u << s;
        const int b = f / n2, r = f - b * n2;
        const int i = r / n;
        bij[s] = pack_bij(b, i, r - i * n);
        rho[s] = reinterpret_cast<const double2 *>(a.rho0)[L.off[b] + r];
      }
    }
  }
  auto valid = [&](int s) { return ((vmask >> s) & 1u) != 0; };
  // pack element index of slot s
  auto flat = [&](int s) {
    if constexpr (COL) return slot_b(bij[s]) * n2 + slot_i(bij[s]) * n + slot_j(bij[s]);
    else return tid + s * T;
  };
  auto goff = [&](uint32_t v) { return L.off[slot_b(v)] + slot_i(v) * n + slot_j(v); };
  // the segment whose amplitudes L.u holds: they are loaded again only when
  // a step lies in another segment (the same for every thread)
  int u_seg = -2;
  auto set_u = [&](int st) {  // between two barriers
    const int seg = a.seg_of_step[st];
    if (seg == u_seg) return;
    u_seg = seg;
    for (int idx = tid; idx < m * pk.nb; idx += T) {
      const int b = idx / pk.nb, q = idx - b * pk.nb;
      L.u[idx] = seg >= 0 ? a.u[((int64_t)L.ids[b] * a.n_ctrl + q) * a.n_seg + seg] : 0.0;
    }
  };
  // element of L y (fwd) or L^+ y (adjoint) for slot s; Y holds the input
  auto apply = [&](int s, const double2 &yij, bool adjoint) {
    uint32_t v = bij[s];
    asm volatile("" : "+v"(v));
    const int b = slot_b(v);
    const uint8_t *blob = L.blobs + (size_t)b * pk.blob_stride;
    const OpView op = adjoint ? make_view(blob + pk.fwd_bytes, BA) : make_view(blob, BF);
    if constexpr (COL) {
      uint32_t ri = adjoint ? ria[s] : rif[s];
      asm volatile("" : "+v"(ri));
      return lindblad_col<WO, NC, NQ, true>(op, adjoint ? cda : cdf, L.Y + b * n2, slot_i(v), ri,
                                            slot_j(v), yij, L.u + b * pk.nb);
    } else {
      return lindblad_elem(op, L.Y + b * n2, slot_i(v), slot_j(v), yij, L.u + b * pk.nb);
    }
  };

  // ---- forward pass with checkpoints
  double2 *ck = reinterpret_cast<double2 *>(a.ckpt);
  for (int st = 0; st < a.nsteps; ++st) {
    if (st % a.ckpt_every == 0) {
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) ck[(int64_t)(st / a.ckpt_every) * SE + goff(bij[s])] = rho[s];
    }
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      yn[s] = rho[s];
      acc[s] = make_double2(0.0, 0.0);
    }
    for (int stage = 0; stage < 4; ++stage) {
      const double cnext = stage < 2 ? 0.5 * h : (stage == 2 ? h : 0.0);
      const double wgt = (stage == 0 || stage == 3) ? 1.0 : 2.0;
      __syncthreads();
      if (stage == 0) set_u(st);
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) L.Y[flat(s)] = yn[s];
      __syncthreads();
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) {
          const double2 kv = apply(s, yn[s], false);
          acc[s] = caxpy(wgt, kv, acc[s]);
          yn[s] = caxpy(cnext, kv, rho[s]);
        }
    }
#pragma unroll
    for (int s = 0; s < EPT; ++s) rho[s] = caxpy(h / 6.0, acc[s], rho[s]);
  }

  // ---- cost: J = Re sum_ij O_ij rho_ji ; lambda = O^+
  __syncthreads();
#pragma unroll
  for (int s = 0; s < EPT; ++s)
    if (valid(s)) L.Y[flat(s)] = rho[s];
  __syncthreads();
  const double2 *O = reinterpret_cast<const double2 *>(a.O);
  double2 lam[EPT];
  double part[EPT];
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    lam[s] = make_double2(0.0, 0.0);
    part[s] = 0.0;
    if (valid(s)) {
      const uint32_t v = bij[s];
      const int b = slot_b(v), i = slot_i(v), j = slot_j(v);
      const double2 oij = O[L.off[b] + i * n + j];
      const double2 rji = L.Y[b * n2 + j * n + i];
      part[s] = oij.x * rji.x - oij.y * rji.y;
      lam[s] = cconj(O[L.off[b] + j * n + i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < EPT; ++s)
    if (valid(s)) red[flat(s)] = part[s];
  __syncthreads();
  per_instance_sum<T>(red, m, n2, sums);
  __syncthreads();
  for (int b = tid; b < m; b += T) a.cost[L.ids[b]] = sums[b];

  // ---- backward pass
  const double ck_kap_l[4] = {h / 6.0, h / 3.0, h / 3.0, h / 6.0};
  const double ck_kap_w[4] = {0.5 * h, 0.5 * h, h, 0.0};  // coefficient of w_{i+1}
  double gacc[EPT][NQ];
#pragma unroll
  for (int s = 0; s < EPT; ++s)
#pragma unroll
    for (int q = 0; q < NQ; ++q) gacc[s][q] = 0.0;
  int cur_seg = -1;
  // adds every slot's accumulated gradient of segment cur_seg to grad
  auto flush = [&]() {
    for (int q = 0; q < NQ; ++q) {
      __syncthreads();
#pragma unroll
      for (int s = 0; s < EPT; ++s)
        if (valid(s)) red[flat(s)] = gacc[s][q];
      __syncthreads();
      per_instance_sum<T>(red, m, n2, sums);
      __syncthreads();
      if (cur_seg >= 0)
        for (int b = tid; b < m; b += T)
          a.grad[((int64_t)L.ids[b] * a.n_ctrl + q) * a.n_seg + cur_seg] += sums[b];
    }
#pragma unroll
    for (int s = 0; s < EPT; ++s)
#pragma unroll
      for (int q = 0; q < NQ; ++q) gacc[s][q] = 0.0;
  };
  double2 *SB = reinterpret_cast<double2 *>(a.stages);
  const int n_ck = (a.nsteps + a.ckpt_every - 1) / a.ckpt_every;
  for (int c = n_ck - 1; c >= 0; --c) {
    const int s0 = c * a.ckpt_every, s1 = min(s0 + a.ckpt_every, a.nsteps);
    // recompute the stage inputs of steps s0..s1-1
#pragma unroll
    for (int s = 0; s < EPT; ++s)
      if (valid(s)) rho[s] = ck[(int64_t)c * SE + goff(bij[s])];
    for (int st = s0; st < s1; ++st) {
#pragma unroll
      for (int s = 0; s < EPT; ++s) {
        yn[s] = rho[s];
        acc[s] = make_double2(0.0, 0.0);
      }
      for (int stage = 0; stage < 4; ++stage) {
        const double cnext = stage < 2 ? 0.5 * h : (stage == 2 ? h : 0.0);
        const double wgt = (stage == 0 || stage == 3) ? 1.0 : 2.0;
        __syncthreads();
        if (stage == 0) set_u(st);
#pragma unroll
        for (int s = 0; s < EPT; ++s)
          if (valid(s)) {
            L.Y[flat(s)] = yn[s];
            SB[((int64_t)(st - s0) * 4 + stage) * SE + goff(bij[s])] = yn[s];
          }
        __syncthreads();
        if (stage < 3) {
#pragma unroll
          for (int s = 0; s < EPT; ++s)
            if (valid(s)) {
              const double2 kv = apply(s, yn[s], false);
              acc[s] = caxpy(wgt, kv, acc[s]);
              yn[s] = caxpy(cnext, kv, rho[s]);
            }
        } else {
#pragma unroll
          for (int s = 0; s < EPT; ++s)
            if (valid(s)) acc[s] = caxpy(wgt, apply(s, yn[s], false), acc[s]);
        }
      }
#pragma unroll
      for (int s = 0; s < EPT; ++s) rho[s] = caxpy(h / 6.0, acc[s], rho[s]);
    }
    // step back through the interval; the stage input of the next (earlier)
    // stage is loaded into registers while this stage computes
    double2 sbn[EPT];
#pragma unroll
    for (int s = 0; s < EPT; ++s)
      sbn[s] = valid(s) ? SB[((int64_t)(s1 - 1 - s0) * 4 + 3) * SE + goff(bij[s])]
                        : make_double2(0.0, 0.0);
    for (int st = s1 - 1; st >= s0; --st) {
      const int seg = a.seg_of_step[st];
      if (seg != cur_seg) {
        flush();
        cur_seg = seg;
      }
      // acc: w_{i+1} of the previous stage; yn: sum of the w_i
#pragma unroll
      for (int s = 0; s < EPT; ++s) {
        acc[s] = make_double2(0.0, 0.0);
        yn[s] = make_double2(0.0, 0.0);
      }
      for (int stage = 3; stage >= 0; --stage) {
        double2 kap[EPT];
#pragma unroll
        for (int s = 0; s < EPT; ++s)
          kap[s] = caxpy(ck_kap_w[stage], acc[s],
                         make_double2(ck_kap_l[stage] * lam[s].x, ck_kap_l[stage] * lam[s].y));
        // gradient: Re <kappa_i, B_q Y_i>
        __syncthreads();
        if (stage == 3) set_u(st);
#pragma unroll
        for (int s = 0; s < EPT; ++s)
          if (valid(s)) L.Y[flat(s)] = sbn[s];
        {  // prefetch: stage - 1 of this step, or stage 3 of the step before
          const int pst = stage > 0 ? st : st - 1, pstage = stage > 0 ? stage - 1 : 3;
          if (pst >= s0) {
#pragma unroll
            for (int s = 0; s < EPT; ++s)
              if (valid(s)) sbn[s] = SB[((int64_t)(pst - s0) * 4 + pstage) * SE + goff(bij[s])];
          }
        }
        __syncthreads();
        if (seg >= 0) {
#pragma unroll
          for (int s = 0; s < EPT; ++s)
            if (valid(s)) {
              const uint32_t v = bij[s];
              const int b = slot_b(v), i = slot_i(v), j = slot_j(v);
              const OpView op = make_view(L.blobs + (size_t)b * pk.blob_stride, BF);
              const double2 *Yb = L.Y + b * n2;
              const double2 yij = Yb[i * n + j];
#pragma unroll
              for (int q = 0; q < NQ; ++q) {
                double2 bq;
                if constexpr (COL)
                  bq = control_col<WO, NC, NQ, true>(op, cdf, Yb, Yb + mul24(i, n), i, j, yij, q);
                else
                  bq = two_sided(op.DB + q * n, op.OBval + q * op.wb * n, op.OBcol + q * op.wb * n,
                                 op.wb, n, Yb, i, j, yij);
                gacc[s][q] += kap[s].x * bq.x + kap[s].y * bq.y;
              }
            }
        }
        // w_i = L^+ kappa_i
        __syncthreads();
#pragma unroll
        for (int s = 0; s < EPT; ++s)
          if (valid(s)) L.Y[flat(s)] = kap[s];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < EPT; ++s)
          if (valid(s)) {
            acc[s] = apply(s, kap[s], true);
            yn[s] = cadd(yn[s], acc[s]);
          }
      }
#pragma unroll
      for (int s = 0; s < EPT; ++s) lam[s] = cadd(lam[s], yn[s]);
    }
  }
  flush();
}

// ---------------------------------------------------------------------------
// One application of L (or L^+) to every instance, stage input in LDS.
// ---------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(T) void apply_lds_kernel(ApplyArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const PackDesc pk = a.packs[blockIdx.x];
  const int n = pk.n, n2 = n * n, E = pk.m * n2;
  const PackLds L = carve(smem, pk);
  const BlobLayout BL = blob_layout(n, pk.wo, pk.nb, pk.wb, pk.nc, pk.wc);
  for (int b = threadIdx.x; b < pk.m; b += T) {
    L.ids[b] = a.order[pk.first + b];
    L.off[b] = a.inst[L.ids[b]].rho_off;
  }
  stage_blobs(L.blobs, pk, a.order, a.inst, a.ops, a.adjoint);
  __syncthreads();
  for (int idx = threadIdx.x; idx < pk.m * pk.nb; idx += T) {
    const int b = idx / pk.nb, q = idx - b * pk.nb;
    L.u[idx] = a.seg >= 0 ? a.u[((int64_t)L.ids[b] * a.n_ctrl + q) * a.n_seg + a.seg] : 0.0;
  }
  for (int f = threadIdx.x; f < E; f += T) {
    const int b = f / n2;
    L.Y[f] = reinterpret_cast<const double2 *>(a.y)[L.off[b] + (f - b * n2)];
  }
  __syncthreads();
  for (int f = threadIdx.x; f < E; f += T) {
    const int b = f / n2, r = f - b * n2;
    const int i = r / n, j = r - i * n;
    const OpView op = make_view(L.blobs + (size_t)b * pk.blob_stride, BL);
    const double2 kv = lindblad_elem(op, L.Y + b * n2, i, j, L.Y[f], L.u + b * pk.nb);
    reinterpret_cast<double2 *>(a.out)[L.off[b] + r] = kv;
  }
}

// ---------------------------------------------------------------------------
// One application of L to every instance, operator shape as a template
// (monomial jumps): y staged in LDS with coalesced loads, then each element
// issues all of its operator and gather reads at once (no index-load chains)
// and the result is stored coalesced.  Same arithmetic order as
// lindblad_elem().
// ---------------------------------------------------------------------------
template <int T, int WO, int NC, int NB, bool RE>
__global__ __launch_bounds__(T) void apply_shape_kernel(ApplyArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const PackDesc pk = a.packs[blockIdx.x];
  const int n = pk.n, n2 = n * n, E = pk.m * n2;
  const PackLds L = carve(smem, pk);
  const BlobLayout BL = blob_layout(n, pk.wo, pk.nb, pk.wb, pk.nc, pk.wc);
  for (int b = threadIdx.x; b < pk.m; b += T) {
    L.ids[b] = a.order[pk.first + b];
    L.off[b] = a.inst[L.ids[b]].rho_off;
  }
  stage_blobs(L.blobs, pk, a.order, a.inst, a.ops, a.adjoint);
  __syncthreads();
  for (int idx = threadIdx.x; idx < pk.m * pk.nb; idx += T) {
    const int b = idx / pk.nb, q = idx - b * pk.nb;
    L.u[idx] = a.seg >= 0 ? a.u[((int64_t)L.ids[b] * a.n_ctrl + q) * a.n_seg + a.seg] : 0.0;
  }
  const double2 *y = reinterpret_cast<const double2 *>(a.y);
  for (int f = threadIdx.x; f < E; f += T) {
    const int b = f / n2;
    L.Y[f] = y[L.off[b] + (f - b * n2)];
  }
  __syncthreads();
  double2 *out = reinterpret_cast<double2 *>(a.out);
  for (int f = threadIdx.x; f < E; f += T) {
    const int b = f / n2, r = f - b * n2;
    const int i = r / n, j = r - i * n;
    const OpView op = make_view(L.blobs + (size_t)b * pk.blob_stride, BL);
    ColData<WO, NC, NB> cd;
    load_column<WO, NC, NB>(cd, op, j);
    const uint32_t ri = row_indices<WO, NC>(op, i);
    out[L.off[b] + r] =
        lindblad_col<WO, NC, NB, RE>(op, cd, L.Y + b * n2, i, ri, j, L.Y[f], L.u + b * pk.nb);
  }
}

// ---------------------------------------------------------------------------
// One application of L, column-owner layout (the pack plan of the column
// kernels: thread t < m*n*G owns column j of instance b and rows g, g+G, ...):
// each thread copies its own elements of y into LDS (coalesced along j),
// loads its column's operator data once, then computes and stores its
// elements (coalesced).  No per-element index division.
// ---------------------------------------------------------------------------
template <int T, int WO, int NC, int NB, bool RE>
__global__ __launch_bounds__(T) void apply_col_kernel(ApplyArgs a) {
  using RL = Rec<WO, NC, NB>;
  extern __shared__ __align__(16) uint8_t smem[];
  const PackDesc pk = a.packs[blockIdx.x];
  const int n = pk.n, n2 = n * n, C = pk.m * n, G = pk.G;
  const PackLds L = carve(smem, pk);
  const int tid = threadIdx.x;
  for (int b = tid; b < pk.m; b += T) {
    L.ids[b] = a.order[pk.first + b];
    L.off[b] = a.inst[L.ids[b]].rho_off;
  }
  stage_records<WO, NC, NB>(L.blobs, pk, a.order, a.inst, a.ops, a.adjoint);
  __syncthreads();
  for (int idx = tid; idx < pk.m * pk.nb; idx += T) {
    const int b = idx / pk.nb, q = idx - b * pk.nb;
    L.u[idx] = a.seg >= 0 ? a.u[((int64_t)L.ids[b] * a.n_ctrl + q) * a.n_seg + a.seg] : 0.0;
  }
  const bool active = tid < C * G;
  const int g = active ? tid / C : 0;
  const int c = active ? tid - g * C : 0;
  const int b = c / n, j = c - b * n;
  double2 *Yb = L.Y + b * n2;
  const double2 *y = reinterpret_cast<const double2 *>(a.y) + L.off[b];
  double2 *out = reinterpret_cast<double2 *>(a.out) + L.off[b];
  if (active) {
    // eight loads in flight per lane before the LDS writes
    int i = g;
    for (; i + 7 * G < n; i += 8 * G) {
      double2 t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = y[(i + u * G) * n + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) Yb[(i + u * G) * n + j] = t[u];
    }
    for (; i < n; i += G) Yb[i * n + j] = y[i * n + j];
  }
  __syncthreads();
  if (!active) return;
  const uint32_t yb = (uint32_t)(reinterpret_cast<uint8_t *>(Yb) - smem);
  const uint32_t recb = (uint32_t)(L.blobs + (size_t)b * pk.blob_stride - smem);
  ColPos<WO, NC, NB> cd;
  {
    const InstDesc &d = a.inst[L.ids[b]];
    const OpView gop = make_view(a.ops + (a.adjoint ? d.adj_off : d.ops_off),
                                 blob_layout(n, pk.wo, pk.nb, pk.wb, pk.nc, pk.wc));
    load_column_pos<WO, NC, NB>(cd, gop, j, yb);
  }
  for (int i = g; i < n; i += G)
    out[i * n + j] = lindblad_rec<WO, NC, NB, RE>(smem, recb + i * RL::S, cd, Yb[i * n + j],
                                                  L.u + b * pk.nb, pk.wb);
}

// ---------------------------------------------------------------------------
// Pipelined column application (persistent).  One workgroup per CU walks
// its tiles (blockIdx.x, + gridDim.x, ...) with two LDS stages: while it
// computes and stores tile t from one stage, the loads of its share of the
// next tile (y rows and row records, 16-byte loads into registers) are in
// flight; once its elements of t are done each thread writes that share into
// the other stage; one barrier per tile.  HBM reads of the next tile thus
// overlap the arithmetic and the stores of the current one.  Column data come from the staged row
// records (the record of row j of A holds the column-j entries of A^+ and of
// the jumps), so a tile needs nothing else from memory.
// ---------------------------------------------------------------------------
template <int WO, int NC, int NB>
__device__ __forceinline__ void load_column_staged(ColPos<WO, NC, NB> &cd, const uint8_t *base,
                                                   uint32_t rec, int n, uint32_t yb, int j) {
  using RL = Rec<WO, NC, NB>;
  int32_t hd[RL::H / 4];
#pragma unroll
  for (int t = 0; t < RL::H / 16; ++t) {
    const int4 q = *reinterpret_cast<const int4 *>(base + rec + 16 * t);
    hd[4 * t] = q.x;
    hd[4 * t + 1] = q.y;
    hd[4 * t + 2] = q.z;
    hd[4 * t + 3] = q.w;
  }
  const double2 *v = reinterpret_cast<const double2 *>(base + rec + RL::H);
  // header offsets are row offsets c*n*16; the column offset is c*16
  cd.dj = cconj(v[RL::D]);
  cd.ybj = yb + 16 * j;
#pragma unroll
  for (int w = 0; w < WO; ++w) {
    cd.yo[w] = yb + (uint32_t)hd[1 + w] / (uint32_t)n;
    cd.oval[w] = cconj(v[RL::O + w]);
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    cd.yj[k] = yb + (uint32_t)hd[1 + WO + k] / (uint32_t)n;
    cd.jval[k] = cconj(v[RL::J + k]);
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    cd.dbj[q] = cconj(v[RL::CB + q * RL::CQ]);
#pragma unroll
    for (int w = 0; w < kColWB; ++w) {
      cd.yob[q][w] = yb + (uint32_t)hd[1 + WO + NC + q * kColWB + w] / (uint32_t)n;
      cd.obval[q][w] = cconj(v[RL::CB + q * RL::CQ + 1 + w]);
    }
  }
}

template <int WO, int NC, int NB, bool RE>
__global__ __launch_bounds__(kPipeT) void apply_pipe_kernel(PipeArgs a) {
  using RL = Rec<WO, NC, NB>;
  constexpr int T = kPipeT, U = kPipeUnits;
  typedef unsigned v4u __attribute__((ext_vector_type(4)));
  extern __shared__ __align__(16) uint8_t smem[];
  PTile *desc = reinterpret_cast<PTile *>(smem + 2 * kPipeStage);
  const int tid = threadIdx.x;
  const int nt = a.n_tiles > (int)blockIdx.x
                     ? (a.n_tiles - (int)blockIdx.x + (int)gridDim.x - 1) / (int)gridDim.x
                     : 0;
  if (nt == 0) return;
  // this workgroup's tile descriptors (tiles blockIdx.x + k*gridDim.x) into LDS
  {
    constexpr int W = sizeof(PTile) / 4;
    for (int idx = tid; idx < nt * W; idx += T) {
      const int k = idx / W, w = idx - k * W;
      reinterpret_cast<int32_t *>(desc + k)[w] = reinterpret_cast<const int32_t *>(
          a.tiles + blockIdx.x + (int64_t)k * gridDim.x)[w];
    }
  }

  // this thread's 16-byte units of a tile: y units first, then records
  const v4u *__restrict__ yv = reinterpret_cast<const v4u *>(a.y);
  const uint8_t *__restrict__ recs = a.recs;
  v4u pf[U];
  auto fetch = [&](const PTile *tl) {
    const int n = tl->n, m = tl->m, h0 = tl->h0;
    const int per = tl->span * n, Ey = m * per;
    const int ru = n * RL::S / 16, Er = m * ru;
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int e = tid + q * T;
      const bool isy = e < Ey;
      const int r = isy ? e : e - Ey, d = isy ? per : ru;
      const int k = min(r / d, m - 1), rem = r - k * d;
      // streaming (non-temporal) loads; past the tile's units the load
      // repeats the tile's first unit
      const bool live = e < Ey + Er;
      const v4u *src = isy    ? yv + tl->yoff[k] + (int64_t)h0 * n + rem
                       : live ? reinterpret_cast<const v4u *>(recs + tl->roff[k]) + rem
                              : yv + tl->yoff[0] + (int64_t)h0 * n;
      pf[q] = __builtin_nontemporal_load(src);
    }
  };
  // every unit is written (units past the tile go to a spare 16 bytes past
  // the descriptor table), so no load is left pending on any path
  uint8_t *spare = smem + 2 * kPipeStage + kPipeMaxTiles * (int)sizeof(PTile);
  auto place = [&](const PTile *tl, uint8_t *stage) {
    const int Ey = tl->m * tl->span * tl->n, Er = tl->m * tl->n * RL::S / 16;
    const int rec_lds = tl->rec_lds;
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int e = tid + q * T;
      uint8_t *dst = e < Ey ? stage + 16 * e
                     : e - Ey < Er ? stage + rec_lds + 16 * (e - Ey) : spare;
      *reinterpret_cast<v4u *>(dst) = pf[q];
    }
  };
  // per-thread global data of a tile (read before the next tile's loads are
  // issued, so that the arithmetic never waits on those)
  struct Prep {
    double2 *out;
    double uq[NB > 0 ? NB : 1];
  };
  auto prep = [&](const PTile *tl) {
    Prep p;
    const int C = tl->m * tl->n;
    const int b = tid < C * tl->G ? (tid % C) / tl->n : 0;
    p.out = reinterpret_cast<double2 *>(a.out) + tl->yoff[b];
#pragma unroll
    for (int q = 0; q < NB; ++q)
      p.uq[q] = a.seg >= 0 ? a.u[((int64_t)tl->id[b] * a.n_ctrl + q) * a.n_seg + a.seg] : 0.0;
    return p;
  };
  auto compute = [&](const PTile *tl, const uint8_t *stage, const Prep &p) {
    const int n = tl->n, C = tl->m * n, G = tl->G, r0 = tl->r0, r1 = tl->r1, wb = tl->wb;
    if (tid >= C * G) return;
    const int g = tid / C, c = tid - g * C, b = c / n, j = c - b * n;
    // LDS address of row 0 of instance b (the stage holds rows h0 ..)
    const uint32_t yb = (uint32_t)(stage - smem) + 16u * (uint32_t)(b * tl->span * n) -
                        16u * (uint32_t)(tl->h0 * n);
    const uint32_t rb = (uint32_t)(stage - smem) + tl->rec_lds + b * n * RL::S;
    ColPos<WO, NC, NB> cd;
    load_column_staged<WO, NC, NB>(cd, smem, rb + j * RL::S, n, yb, j);
    for (int i = r0 + g; i < r1; i += G) {
      const double2 yij = *reinterpret_cast<const double2 *>(smem + yb + 16 * (i * n + j));
      p.out[i * n + j] = lindblad_rec<WO, NC, NB, RE>(smem, rb + i * RL::S, cd, yij, p.uq, wb);
    }
  };

  __syncthreads();
  fetch(desc);
  place(desc, smem);
  int s = 0;
  for (int k = 0;; ++k) {
    __syncthreads();  // stage s holds tile k; every thread is done with stage s^1
    const Prep p = prep(desc + k);
    if (k + 1 >= nt) {
      compute(desc + k, smem + s * kPipeStage, p);
      break;
    }
    fetch(desc + k + 1);
    compute(desc + k, smem + s * kPipeStage, p);
    place(desc + k + 1, smem + (s ^ 1) * kPipeStage);
    s ^= 1;
  }
}

// ---------------------------------------------------------------------------
// Streamed Liouvillian application: y and out in HBM, operators read through
// the caches.  A workgroup takes one tile (a contiguous element range of one
// instance); thread t handles elements e0 + t, e0 + t + T, ...: consecutive
// lanes take consecutive columns, so the row gathers y[col][j], the output
// stores and the j-side operator reads are coalesced, and the i-side reads
// are shared by the lanes of a row.
// ---------------------------------------------------------------------------
// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with its own L2; workgroup w runs tile (w mod 8) * ceil(n_tiles/8) + w / 8,
// so every XCD walks a contiguous eighth of the batch and the neighbouring
// rows an instance's gathers touch stay in one L2.
__device__ __forceinline__ int xcd_tile(int n_tiles) {
  const int per = (n_tiles + 7) / 8;
  return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

template <int T>
__global__ __launch_bounds__(T) void apply_global_kernel(ApplyGArgs a) {
  // tiles are fixed 2048-element chunks of the packed state buffer and may
  // span several instances; e0/e1 are packed offsets, inst the first instance
  const int tix = xcd_tile(a.n_tiles);
  if (tix >= a.n_tiles) return;
  const Tile tl = a.tiles[tix];
  const double2 *Y = reinterpret_cast<const double2 *>(a.y);
  double2 *out = reinterpret_cast<double2 *>(a.out);
  int b = tl.inst;
  int64_t lo = a.inst[b].rho_off, hi = lo + (int64_t)a.inst[b].n * a.inst[b].n;
  for (int64_t g = tl.e0 + threadIdx.x; g < tl.e1; g += T) {
    while (g >= hi) {  // next instance (monotone)
      ++b;
      lo = hi;
      hi = lo + (int64_t)a.inst[b].n * a.inst[b].n;
    }
    const InstDesc &d = a.inst[b];
    const int n = d.n;
    const Signature &sg = a.adjoint ? d.adj : d.fwd;
    OpView op = make_view(a.ops + (a.adjoint ? d.adj_off : d.ops_off),
                          blob_layout(n, sg.wo, sg.nb, sg.wb, sg.nc, sg.wc));
    if (a.seg < 0) op.nb = 0;  // no control amplitude outside all segments
    const double *uq = a.u + (int64_t)b * a.n_ctrl * a.n_seg + (a.seg < 0 ? 0 : a.seg);
    const int e = (int)(g - lo);
    const int i = e / n, j = e - i * n;
    out[g] = lindblad_elem(op, Y + lo, i, j, Y[g], uq, a.n_seg);
  }
}

// ---------------------------------------------------------------------------
// Row-block streamed application, for instances too large for a resident
// pack (128 <= n <= 1024).  A workgroup takes rows [r0, r1) (at most R) of
// one instance and stages them in LDS; thread t owns columns t, t + 256, ...
// and keeps the R accumulators of its column in registers.  The column side
// of every product (y A^+), and every left product or jump whose source row
// lies in the block, reads LDS; the other source rows are read through the
// caches (the row is the same for the whole workgroup, so each such read is
// one contiguous row segment).  The row-side operator entries are the same
// for all lanes (scalar loads).  Every element accumulates its terms in the
// order of lindblad_elem(), with exactly-zero parts skipped under RE (real
// jump coefficients, imaginary off-diagonal entries), so the results are
// those of the other application kernels.
// ---------------------------------------------------------------------------
// rows per thread of the 16-row kernels
constexpr int kRowsRT = 4;
// Word 3 of a buffer resource for plain (untyped, raw) loads on this chip.
constexpr int kBufferFlags = 0x00020000;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Row-side operator entries are read through the constant address space
// (the same address in every lane: scalar loads, batched by the compiler).
template <typename T>
using cptr = const T __attribute__((address_space(4))) *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)p;
}
__device__ __forceinline__ cptr<double> as_const2(const double2 *p) {
  return (cptr<double>)p;
}
// complex element idx of a constant-space complex array
__device__ __forceinline__ double2 cld(cptr<double> p, int idx) {
  return make_double2(p[2 * idx], p[2 * idx + 1]);
}

// LDS of a row block: the block's rows of y, then the row-side entries of
// its rows: D [R] | Oval [wo][R] | Jval [nc wc][R] (complex) | Ocol [wo][R] |
// Jcol [nc wc][R] (int).
template <int R>
struct RowBlock {
  double2 *Ys, *Rd, *Rov, *Rjv;
  int32_t *Roc, *Rjc;
  int r0, rows;
};

template <int R>
__device__ __forceinline__ RowBlock<R> carve_rows(uint8_t *smem, const OpView &op, int r0,
                                                  int rows) {
  RowBlock<R> k;
  const int n = op.n, ncw = op.nc * op.wc;
  k.Ys = reinterpret_cast<double2 *>(smem);
  k.Rd = k.Ys + R * n;
  k.Rov = k.Rd + R;
  k.Rjv = k.Rov + op.wo * R;
  k.Roc = reinterpret_cast<int32_t *>(k.Rjv + ncw * R);
  k.Rjc = k.Roc + op.wo * R;
  k.r0 = r0;
  k.rows = rows;
  return k;
}

// Stages rows [r0, r0 + rows) of y (n x n, HBM) and their operator entries;
// all NT threads take part, the caller synchronises.
template <int R, int NT>
__device__ __forceinline__ void stage_rows(const RowBlock<R> &k, const OpView &op,
                                           const double2 *Yg) {
  const int n = op.n, ncw = op.nc * op.wc, r0 = k.r0, rows = k.rows;
  for (int e = threadIdx.x; e < rows * n; e += NT) k.Ys[e] = Yg[(int64_t)r0 * n + e];
  for (int e = threadIdx.x; e < (1 + op.wo + ncw) * R; e += NT) {
    const int q = e / R, r = e - q * R;
    if (r >= rows) continue;
    if (q == 0) {
      k.Rd[r] = op.D[r0 + r];
    } else if (q <= op.wo) {
      k.Rov[(q - 1) * R + r] = op.Oval[(q - 1) * n + r0 + r];
      k.Roc[(q - 1) * R + r] = op.Ocol[(q - 1) * n + r0 + r];
    } else {
      const int kk = q - 1 - op.wo;
      k.Rjv[kk * R + r] = op.Jval[kk * n + r0 + r];
      k.Rjc[kk * R + r] = op.Jcol[kk * n + r0 + r];
    }
  }
}

// (L y)_ij for column j and the rows rb + r (r < RT) of a staged block: the
// terms of lindblad_elem() in its order, exactly-zero parts skipped under RE
// (real jump coefficients, imaginary off-diagonal entries).  Source rows
// outside the block are read from Yg (a buffer load over the instance's n^2
// elements: a load kind of its own, so LDS and HBM reads never merge into a
// flat access).  uq[q * ustride] are the control amplitudes (nb of them).
template <int R, int RT, bool RE>
__device__ __forceinline__ void rows_lindblad(const RowBlock<R> &k, const OpView &op,
                                              const double2 *Yg, int nb, const double *uq,
                                              int ustride, int rb, int j, double2 (&acc)[RT]) {
  const int n = op.n, r0 = k.r0, rows = k.rows;
  const double2 *Ys = k.Ys;
  const __amdgpu_buffer_rsrc_t yrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double2 *>(Yg), 0, 16 * n * n, kBufferFlags);
  // element (c, j) of y for a source row c that is the same for all lanes
  auto Yrow = [&](int c, int jj) {
    if (c >= r0 && c < r0 + rows) return Ys[(c - r0) * n + jj];
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(yrs, (uint32_t)(c * n + jj) * 16u, 0, 0);
    return __builtin_bit_cast(double2, v);
  };
  // acc += v * y and acc += conj(v) * y
  auto fma_v = [](double2 v, double2 y, double2 a) {
    if (RE) return make_double2(fma(-v.y, y.y, a.x), fma(v.y, y.x, a.y));
    return cfma(v, y, a);
  };
  auto fma_cv = [](double2 v, double2 y, double2 a) {
    if (RE) return make_double2(fma(v.y, y.y, a.x), fma(-v.y, y.x, a.y));
    return cfma_conj(v, y, a);
  };
  double2 yv[RT];
  const double2 dj = cconj(op.D[j]);
#pragma unroll
  for (int r = 0; r < RT; ++r)
    if (rb + r < rows) acc[r] = cmul(cadd(k.Rd[rb + r], dj), Ys[(rb + r) * n + j]);
  // A y: source rows Ocol[w][i]; the RT gathers of a term are issued before
  // its products
  for (int w = 0; w < op.wo; ++w) {
#pragma unroll
    for (int r = 0; r < RT; ++r)
      if (rb + r < rows) yv[r] = Yrow(k.Roc[w * R + rb + r], j);
#pragma unroll
    for (int r = 0; r < RT; ++r)
      if (rb + r < rows) acc[r] = fma_v(k.Rov[w * R + rb + r], yv[r], acc[r]);
  }
  // y A^+: row i, columns Ocol[w][j]
  for (int w = 0; w < op.wo; ++w) {
    const int c = op.Ocol[w * n + j];
    const double2 v = op.Oval[w * n + j];
#pragma unroll
    for (int r = 0; r < RT; ++r)
      if (rb + r < rows) acc[r] = fma_cv(v, Ys[(rb + r) * n + c], acc[r]);
  }
  // control terms u_q (B_q y + y B_q^+), a separate sum scaled by u_q (row
  // side read through the constant address space)
  for (int q = 0; q < nb; ++q) {
    const double u = uq[q * ustride];
    if (u == 0.0) continue;
    const cptr<double> DBr = as_const2(op.DB + q * n), OBvr = as_const2(op.OBval + q * op.wb * n);
    const cptr<int32_t> OBcr = as_const(op.OBcol + q * op.wb * n);
    const double2 *OBv = op.OBval + q * op.wb * n;
    const int32_t *OBc = op.OBcol + q * op.wb * n;
    double2 t[RT];
    const double2 dbj = cconj(op.DB[q * n + j]);
#pragma unroll
    for (int r = 0; r < RT; ++r)
      if (rb + r < rows) t[r] = cmul(cadd(cld(DBr, r0 + rb + r), dbj), Ys[(rb + r) * n + j]);
    for (int w = 0; w < op.wb; ++w) {
#pragma unroll
      for (int r = 0; r < RT; ++r)
        if (rb + r < rows) yv[r] = Yrow(OBcr[w * n + r0 + rb + r], j);
#pragma unroll
      for (int r = 0; r < RT; ++r)
        if (rb + r < rows) t[r] = fma_v(cld(OBvr, w * n + r0 + rb + r), yv[r], t[r]);
    }
    for (int w = 0; w < op.wb; ++w) {
      const int c = OBc[w * n + j];
      const double2 v = OBv[w * n + j];
#pragma unroll
      for (int r = 0; r < RT; ++r)
        if (rb + r < rows) t[r] = fma_cv(v, Ys[(rb + r) * n + c], t[r]);
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
      if (rb + r < rows) acc[r] = caxpy(u, t[r], acc[r]);
  }
  // jumps C_k y C_k^+
  for (int kk = 0; kk < op.nc; ++kk) {
    const int kw = kk * op.wc * n;
    for (int w = 0; w < op.wc; ++w)
      for (int v = 0; v < op.wc; ++v) {
        const double2 vj = op.Jval[kw + v * n + j];
        const int cj = op.Jcol[kw + v * n + j];
        const int slot = (kk * op.wc + w) * R + rb;
#pragma unroll
        for (int r = 0; r < RT; ++r)
          if (rb + r < rows) yv[r] = Yrow(k.Rjc[slot + r], cj);
#pragma unroll
        for (int r = 0; r < RT; ++r)
          if (rb + r < rows) {
            const double2 vi = k.Rjv[slot + r];
            if (RE) {
              const double p = vi.x * vj.x;
              acc[r] = make_double2(fma(p, yv[r].x, acc[r].x), fma(p, yv[r].y, acc[r].y));
            } else {
              acc[r] = cfma(cmul(vi, cconj(vj)), yv[r], acc[r]);
            }
          }
      }
  }
}

// Two workgroups per CU (8 wavefronts per SIMD, at most 64 VGPRs): the
// kernel waits on its remote-row loads, and the extra wavefronts hide that
// latency better than the registers the cap spills cost.
template <int R, int RT, bool RE>
__global__ __launch_bounds__(256 * R / RT, 8) void apply_rows_kernel(ApplyGArgs a) {
  constexpr int NT = 256 * R / RT;  // threads: 256 columns x R / RT row groups
  extern __shared__ __align__(16) uint8_t smem[];
  const int tix = xcd_tile(a.n_tiles);
  if (tix >= a.n_tiles) return;
  const Tile tl = a.tiles[tix];
  const int b = tl.inst;
  const InstDesc &d = a.inst[b];
  const int n = d.n;
  const Signature &sg = a.adjoint ? d.adj : d.fwd;
  const OpView op = make_view(a.ops + (a.adjoint ? d.adj_off : d.ops_off),
                              blob_layout(n, sg.wo, sg.nb, sg.wb, sg.nc, sg.wc));
  const int nb = a.seg < 0 ? 0 : op.nb;  // no control amplitude outside all segments
  const double *uq = a.u + (int64_t)b * a.n_ctrl * a.n_seg + (a.seg < 0 ? 0 : a.seg);
  const double2 *Yg = reinterpret_cast<const double2 *>(a.y) + d.rho_off;
  double2 *out = reinterpret_cast<double2 *>(a.out) + d.rho_off;
  const RowBlock<R> k = carve_rows<R>(smem, op, tl.e0, tl.e1 - tl.e0);
  stage_rows<R, NT>(k, op, Yg);
  __syncthreads();
  // this thread's rows rb + r, r < RT (the same for the whole wavefront)
  const int rb = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 256) * RT);
  for (int j = (int)(threadIdx.x & 255); j < n; j += 256) {
    double2 acc[RT];
    rows_lindblad<R, RT, RE>(k, op, Yg, nb, uq, a.n_seg, rb, j, acc);
#pragma unroll
    for (int r = 0; r < RT; ++r)
      if (rb + r < k.rows) out[(int64_t)(k.r0 + rb + r) * n + j] = acc[r];
  }
}

// ---------------------------------------------------------------------------
// Superoperator form: out = S y with S the explicit n^2 x n^2 Liouvillian of
// each instance in slot-major ELL (consecutive rows adjacent per slot, so the
// column and value reads are coalesced); y read through the caches.
// ---------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(T) void superop_kernel(SuperArgs a) {
  const int tix = xcd_tile(a.n_tiles);
  if (tix >= a.n_tiles) return;
  const Tile tl = a.tiles[tix];
  const InstDesc &d = a.inst[tl.inst];
  const SuperDesc sd = a.sd[tl.inst];
  const int n2 = d.n * d.n;
  const int32_t *col = a.col + sd.col_off;
  const double2 *val = reinterpret_cast<const double2 *>(a.val) + sd.val_off;
  const double2 *Y = reinterpret_cast<const double2 *>(a.y) + d.rho_off;
  double2 *out = reinterpret_cast<double2 *>(a.out) + d.rho_off;
  for (int e = tl.e0 + threadIdx.x; e < tl.e1; e += T) {
    double2 acc = make_double2(0.0, 0.0);
    for (int s = 0; s < sd.w; ++s) acc = cfma(val[(int64_t)s * n2 + e], Y[col[(int64_t)s * n2 + e]], acc);
    out[e] = acc;
  }
}

// ---------------------------------------------------------------------------
// Streamed steppers: one grid-wide kernel per stage over element tiles
// (XCD-aware order), state and stage data in HBM, operators read through the
// caches.  Used when an instance's state does not fit in LDS.  The adaptive
// stepper keeps each instance's control (DpCtl) in HBM: the stage kernels skip
// finished instances, a single-workgroup control kernel reduces the tile
// partial error sums of every instance in a fixed order and takes the same
// decisions as the resident kernel.
// ---------------------------------------------------------------------------

// Controller decision after an attempted step (same rule as the resident
// kernel) followed by the set-up of the next attempt.
__device__ void dp_decide_and_setup(DpCtl &c, double err, const StreamArgs &a) {
  c.accept = 0;
  c.k1_seg = c.seg;
  if (!isfinite(err)) {
    c.status = 5;  // LME_ENONFINITE
    c.active = 0;
  } else if (err <= 1.0) {
    c.accept = 1;
    ++c.n_acc;
    double fac = (err == 0.0) ? 10.0 : 0.9 * pow(err, -0.2);
    fac = fmin(10.0, fmax(0.2, fac));
    if (c.prev_rej && fac > 1.0) fac = 1.0;
    c.prev_rej = 0;
    c.h = c.h_try * fac;
    if (c.landing) {
      c.t = a.stops[c.stop];
      c.out_due = a.stop_out[c.stop];
      if (++c.stop == a.n_stops) c.active = 0;
    } else {
      c.t += c.h_try;
    }
  } else {
    ++c.n_rej;
    c.prev_rej = 1;
    c.h = c.h_try * fmax(0.2, 0.9 * pow(err, -0.2));
  }
}

__device__ void dp_setup(DpCtl &c, const StreamArgs &a) {
  if (!c.active) return;
  if (c.n_acc + c.n_rej >= a.max_steps) {
    c.status = 3;  // LME_EMAXSTEPS
    c.active = 0;
  } else if (c.h < a.h_min) {
    c.status = 4;  // LME_ESTEPUNDERFLOW
    c.active = 0;
  } else {
    const double ts = a.stops[c.stop];
    c.landing = c.h >= ts - c.t;
    c.h_try = c.landing ? ts - c.t : c.h;
    c.seg = a.n_seg > 0 ? a.stop_seg[c.stop] : -1;
    c.need_k1 = c.k1_seg != c.seg;
  }
}

// Fixed-order sum of one value per thread over the workgroup.
template <int T>
__device__ double block_sum(double v, double *sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < T / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

struct TileCtx {
  int b, n, e0, e1;
  int64_t base;
  OpView op;
};

__device__ __forceinline__ TileCtx tile_ctx(const StreamArgs &a, int tix, double *uq, int seg) {
  const Tile tl = a.tiles[tix];
  const InstDesc &d = a.inst[tl.inst];
  TileCtx t;
  t.b = tl.inst;
  t.n = d.n;
  t.e0 = tl.e0;
  t.e1 = tl.e1;
  t.base = d.rho_off;
  const Signature &sg = d.fwd;
  t.op = make_view(a.ops + d.ops_off, blob_layout(d.n, sg.wo, sg.nb, sg.wb, sg.nc, sg.wc));
  for (int q = threadIdx.x; q < sg.nb; q += blockDim.x)
    uq[q] = seg >= 0 ? a.u[((int64_t)tl.inst * a.n_ctrl + q) * a.n_seg + seg] : 0.0;
  return t;
}

// Stage s (0..6) of the adaptive step: k_s = L(y_s); the input of stage s+1,
// y_{s+1} = rho + h sum_{j<=s} a[s+1][j] k_j, or, after the last stage, the
// partial sum of the squared scaled error of the tile.
//   inputs  y_0 = rho, y_1 = yb0, y_2 = yb1, y_3 = yb0, y_4 = yb1, y_5 = yb0,
//           y_6 = y5 (the fifth-order solution)
template <int T>
__global__ __launch_bounds__(T) void sdp_stage_kernel(StreamArgs a, int s) {
  __shared__ double uq[kMaxWidth];
  __shared__ double sh[T / 64];
  const int tix = xcd_tile(a.n_tiles);
  if (tix >= a.n_tiles) return;
  const int b = a.tiles[tix].inst;
  const DpCtl c = a.ctl[b];
  if (!c.active) return;
  const TileCtx t = tile_ctx(a, tix, uq, c.seg);
  __syncthreads();
  double2 *rho = reinterpret_cast<double2 *>(a.rho) + t.base;
  double2 *yb[2] = {reinterpret_cast<double2 *>(a.yb0) + t.base,
                    reinterpret_cast<double2 *>(a.yb1) + t.base};
  double2 *y5 = reinterpret_cast<double2 *>(a.y5) + t.base;
  double2 *K = reinterpret_cast<double2 *>(a.K) + t.base;
  const int64_t SE = a.state_elems;
  const double2 *Yin = s == 0 ? rho : (s == 6 ? y5 : yb[(s + 1) & 1]);
  double2 *Yout = s == 5 ? y5 : yb[s & 1];
  double part = 0.0;
  for (int e = t.e0 + threadIdx.x; e < t.e1; e += T) {
    const int i = e / t.n, j = e - i * t.n;
    double2 k;
    if (s > 0 || c.need_k1) {
      k = lindblad_elem(t.op, Yin, i, j, Yin[e], uq);
      K[s * SE + e] = k;
    } else {
      k = K[e];
    }
    if (s < 6) {
      double2 acc = make_double2(0.0, 0.0);
      for (int jj = 0; jj <= s; ++jj) acc = caxpy(kDpA[s + 1][jj], jj == s ? k : K[jj * SE + e], acc);
      Yout[e] = caxpy(c.h_try, acc, rho[e]);
    } else {
      double2 er = make_double2(0.0, 0.0);
      for (int jj = 0; jj < 7; ++jj) er = caxpy(kDpE[jj], jj == 6 ? k : K[jj * SE + e], er);
      er = make_double2(c.h_try * er.x, c.h_try * er.y);
      const double sc = a.atol + a.rtol * fmax(hypot(rho[e].x, rho[e].y), hypot(y5[e].x, y5[e].y));
      const double r = hypot(er.x, er.y) / sc;
      part += r * r;
    }
  }
  if (s == 6) {
    const double tot = block_sum<T>(part, sh);
    if (threadIdx.x == 0) a.tile_part[tix] = tot;
  }
}

// The same stage for batches of row-block tiles (every instance
// 128 <= n <= 256, tiles of at most R whole rows): the stage input's rows
// and their operator entries are staged in LDS and L(y_s) is evaluated by
// rows_lindblad(), then every element of the tile continues as above.
template <int R, int RT, bool RE>
__global__ __launch_bounds__(256 * R / RT, 8) void sdp_stage_rows_kernel(StreamArgs a, int s) {
  constexpr int NT = 256 * R / RT;
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ double uq[kMaxWidth];
  __shared__ double sh[NT / 64];
  const int tix = xcd_tile(a.n_tiles);
  if (tix >= a.n_tiles) return;
  const int b = a.tiles[tix].inst;
  const DpCtl c = a.ctl[b];
  if (!c.active) return;
  const TileCtx t = tile_ctx(a, tix, uq, c.seg);
  double2 *rho = reinterpret_cast<double2 *>(a.rho) + t.base;
  double2 *yb[2] = {reinterpret_cast<double2 *>(a.yb0) + t.base,
                    reinterpret_cast<double2 *>(a.yb1) + t.base};
  double2 *y5 = reinterpret_cast<double2 *>(a.y5) + t.base;
  double2 *K = reinterpret_cast<double2 *>(a.K) + t.base;
  const int64_t SE = a.state_elems;
  const double2 *Yin = s == 0 ? rho : (s == 6 ? y5 : yb[(s + 1) & 1]);
  double2 *Yout = s == 5 ? y5 : yb[s & 1];
  const int n = t.n;
  const bool need = s > 0 || c.need_k1;
  const RowBlock<R> k = carve_rows<R>(smem, t.op, t.e0 / n, (t.e1 - t.e0) / n);
  if (need) stage_rows<R, NT>(k, t.op, Yin);
  __syncthreads();
  const int rb = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 256) * RT);
  double part = 0.0;
  for (int j = (int)(threadIdx.x & 255); j < n; j += 256) {
    double2 kv[RT];
    if (need) rows_lindblad<R, RT, RE>(k, t.op, Yin, t.op.nb, uq, 1, rb, j, kv);
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      if (rb + r >= k.rows) continue;
      const int e = (k.r0 + rb + r) * n + j;
      double2 kk;
      if (need) {
        kk = kv[r];
        K[s * SE + e] = kk;
      } else {
        kk = K[e];
      }
      if (s < 6) {
        double2 acc = make_double2(0.0, 0.0);
        for (int jj = 0; jj <= s; ++jj) acc = caxpy(kDpA[s + 1][jj], jj == s ? kk : K[jj * SE + e], acc);
        Yout[e] = caxpy(c.h_try, acc, rho[e]);
      } else {
        double2 er = make_double2(0.0, 0.0);
        for (int jj = 0; jj < 7; ++jj) er = caxpy(kDpE[jj], jj == 6 ? kk : K[jj * SE + e], er);
        er = make_double2(c.h_try * er.x, c.h_try * er.y);
        const double sc = a.atol + a.rtol * fmax(hypot(rho[e].x, rho[e].y), hypot(y5[e].x, y5[e].y));
        const double q = hypot(er.x, er.y) / sc;
        part += q * q;
      }
    }
  }
  if (s == 6) {
    const double tot = block_sum<NT>(part, sh);
    if (threadIdx.x == 0) a.tile_part[tix] = tot;
  }
}

// Accept / reject for every instance and set-up of its next attempt; one
// workgroup, instances strided over its threads; writes the active count.
template <int T>
__global__ __launch_bounds__(T) void sdp_control_kernel(StreamArgs a) {
  __shared__ double sh[T / 64];
  int act = 0;
  for (int b = threadIdx.x; b < a.n_inst; b += T) {
    DpCtl c = a.ctl[b];
    if (c.active) {
      double sum = 0.0;
      for (int q = 0; q < a.tile_count[b]; ++q) sum += a.tile_part[a.tile_first[b] + q];
      const int n = a.inst[b].n;
      dp_decide_and_setup(c, sqrt(sum / ((double)n * n)), a);
      dp_setup(c, a);
      a.ctl[b] = c;
    } else {
      a.ctl[b].accept = 0;
    }
    act += a.ctl[b].active;
  }
  const double tot = block_sum<T>((double)act, sh);
  if (threadIdx.x == 0) *a.n_active = (int32_t)tot;
}

// Accepted instances move to the fifth-order solution; k7 becomes k1.
template <int T>
__global__ __launch_bounds__(T) void sdp_accept_kernel(StreamArgs a) {
  const int tix = xcd_tile(a.n_tiles);
  if (tix >= a.n_tiles) return;
  const Tile tl = a.tiles[tix];
  if (!a.ctl[tl.inst].accept) return;
  const int64_t base = a.inst[tl.inst].rho_off;
  double2 *rho = reinterpret_cast<double2 *>(a.rho) + base;
  const double2 *y5 = reinterpret_cast<const double2 *>(a.y5) + base;
  double2 *K = reinterpret_cast<double2 *>(a.K) + base;
  for (int e = tl.e0 + threadIdx.x; e < tl.e1; e += T) {
    rho[e] = y5[e];
    K[e] = K[6 * a.state_elems + e];
  }
}

// Outputs of instances whose out_due >= 0 (one workgroup per instance): the
// expectation values (waves over operators, lanes over rows, butterfly) and
// the state; then clears out_due.
template <int T>
__device__ void instance_outputs(const StreamArgs &a, int b, int k, bool check) {
  const InstDesc &d = a.inst[b];
  const int n = d.n, we = d.we;
  const double2 *rho = reinterpret_cast<const double2 *>(a.rho) + d.rho_off;
  if (a.expect && a.n_e > 0) {
    const int32_t *Ec = reinterpret_cast<const int32_t *>(a.eops + d.eops_off);
    const double2 *Ev = reinterpret_cast<const double2 *>(
        a.eops + d.eops_off + eops_val_offset(n, we, a.n_e));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = wave; e < a.n_e; e += T / 64) {
      double2 part = make_double2(0.0, 0.0);
      for (int i = lane; i < n; i += 64)
        for (int w = 0; w < we; ++w) {
          const int idx = (e * we + w) * n + i;
          part = cfma(Ev[idx], rho[Ec[idx] * n + i], part);
        }
      part = wave_sum(part);
      if (lane == 0) {
        double *dst = a.expect + 2 * (((int64_t)b * a.n_e + e) * a.n_t + k);
        dst[0] = part.x;
        dst[1] = part.y;
        if (check && !cfinite(part) && a.status) a.status[b] = 5;  // LME_ENONFINITE
      }
    }
  }
  if (a.states) {
    double2 *st = reinterpret_cast<double2 *>(a.states) + (int64_t)k * a.state_elems + d.rho_off;
    for (int e = threadIdx.x; e < n * n; e += T) st[e] = rho[e];
  }
}

// Outputs of the adaptive stepper: instances whose out_due >= 0 (one
// workgroup per instance), then out_due is cleared.  fixed_k >= 0 writes
// output fixed_k of every instance (the initial state).
template <int T>
__global__ __launch_bounds__(T) void stream_output_kernel(StreamArgs a, int fixed_k) {
  const int b = blockIdx.x;
  const int k = fixed_k >= 0 ? fixed_k : a.ctl[b].out_due;
  if (k < 0) return;
  instance_outputs<T>(a, b, k, fixed_k >= 0);
  __syncthreads();
  if (threadIdx.x == 0 && fixed_k < 0) a.ctl[b].out_due = -1;
}

// ---- streamed fixed-step RK4 ------------------------------------------------
// counters[0] = completed steps, counters[1] = next output index; kernels of a
// step past nsteps return at once, so a graph of several steps may overrun.

// Stage s of RK4: k = L(y_s) with y_0 = rho, y_1 = yb0, y_2 = yb1, y_3 = yb0;
// the accumulator k1 + 2k2 + 2k3 (+ k4) and the next input (or the update of
// rho) in the same operation order as the resident kernels.
template <int T>
__global__ __launch_bounds__(T) void srk_stage_kernel(StreamArgs a, int s) {
  __shared__ double uq[kMaxWidth];
  const int st = a.counters[0];
  if (st >= a.nsteps) return;
  const int tix = xcd_tile(a.n_tiles);
  if (tix >= a.n_tiles) return;
  const TileCtx t = tile_ctx(a, tix, uq, a.seg_of_step[st]);
  __syncthreads();
  double2 *rho = reinterpret_cast<double2 *>(a.rho) + t.base;
  double2 *acc = reinterpret_cast<double2 *>(a.acc) + t.base;
  double2 *yb[2] = {reinterpret_cast<double2 *>(a.yb0) + t.base,
                    reinterpret_cast<double2 *>(a.yb1) + t.base};
  const double2 *Yin = s == 0 ? rho : yb[(s + 1) & 1];
  double2 *Yout = yb[s & 1];
  const double h = a.h;
  const double cnext = s < 2 ? 0.5 * h : h;
  const double wgt = (s == 0 || s == 3) ? 1.0 : 2.0;
  for (int e = t.e0 + threadIdx.x; e < t.e1; e += T) {
    const int i = e / t.n, j = e - i * t.n;
    const double2 k = lindblad_elem(t.op, Yin, i, j, Yin[e], uq);
    const double2 ac = caxpy(wgt, k, s == 0 ? make_double2(0.0, 0.0) : acc[e]);
    if (s < 3) {
      acc[e] = ac;
      Yout[e] = caxpy(cnext, k, rho[e]);
    } else {
      rho[e] = caxpy(h / 6.0, ac, rho[e]);
    }
  }
}

// Outputs due after the step just completed (one workgroup per instance).
template <int T>
__global__ __launch_bounds__(T) void srk_output_kernel(StreamArgs a) {
  const int st = a.counters[0], k = a.counters[1];
  if (st >= a.nsteps || k >= a.n_t || a.out_step[k] != st + 1) return;
  instance_outputs<T>(a, blockIdx.x, k, true);
}

// Advances the counters after a step (one thread); mode 1: initialise them
// (and the status) before the first step.
__global__ void srk_tail_kernel(StreamArgs a, int mode) {
  if (mode == 1) {
    a.counters[0] = 0;
    a.counters[1] = (a.n_t > 0 && a.out_step[0] == 0) ? 1 : 0;
    for (int b = 0; b < a.n_inst && a.status; ++b) a.status[b] = 0;
    return;
  }
  if (mode == 2) {  // counts after the last step
    for (int b = 0; b < a.n_inst && a.counts; ++b) {
      a.counts[2 * (int64_t)b] = a.nsteps;
      a.counts[2 * (int64_t)b + 1] = 0;
    }
    return;
  }
  const int st = a.counters[0];
  if (st >= a.nsteps) return;
  const int k = a.counters[1];
  if (k < a.n_t && a.out_step[k] == st + 1) a.counters[1] = k + 1;
  a.counters[0] = st + 1;
}

// Initial control state of every instance (single workgroup).
template <int T>
__global__ __launch_bounds__(T) void sdp_init_kernel(StreamArgs a) {
  for (int b = threadIdx.x; b < a.n_inst; b += T) {
    DpCtl c;
    c.t = a.t0;
    c.h = a.h0;
    c.h_try = c.hs = 0.0;
    c.n_acc = c.n_rej = 0;
    c.stop = 0;
    c.status = 0;
    c.active = a.n_stops > 0;
    c.accept = c.landing = 0;
    c.seg = -1;
    c.k1_seg = -2;
    c.prev_rej = 0;
    c.out_due = 0;
    c.need_k1 = 1;
    a.ctl[b] = c;
  }
}

// Starting step, part 1 (tiles): f0 = L(rho) with the first interval's
// controls into k1; partial sums of |rho/sc|^2 and |f0/sc|^2.
template <int T>
__global__ __launch_bounds__(T) void sdp_hnw1_kernel(StreamArgs a) {
  __shared__ double uq[kMaxWidth];
  __shared__ double sh[T / 64];
  const int tix = xcd_tile(a.n_tiles);
  if (tix >= a.n_tiles) return;
  const int seg0 = a.n_seg > 0 ? a.stop_seg[0] : -1;
  const TileCtx t = tile_ctx(a, tix, uq, seg0);
  __syncthreads();
  const double2 *rho = reinterpret_cast<const double2 *>(a.rho) + t.base;
  double2 *K = reinterpret_cast<double2 *>(a.K) + t.base;
  double p0 = 0.0, p1 = 0.0;
  for (int e = t.e0 + threadIdx.x; e < t.e1; e += T) {
    const int i = e / t.n, j = e - i * t.n;
    const double2 f0 = lindblad_elem(t.op, rho, i, j, rho[e], uq);
    K[e] = f0;
    const double sc = a.atol + a.rtol * hypot(rho[e].x, rho[e].y);
    const double r0 = hypot(rho[e].x, rho[e].y) / sc, r1 = hypot(f0.x, f0.y) / sc;
    p0 += r0 * r0;
    p1 += r1 * r1;
  }
  const double s0 = block_sum<T>(p0, sh);
  const double s1 = block_sum<T>(p1, sh);
  if (threadIdx.x == 0) {
    a.tile_part[2 * tix] = s0;
    a.tile_part[2 * tix + 1] = s1;
  }
}

// Starting step, part 2 (single workgroup): hs = 0.01 d0/d1 (or 1e-6).
template <int T>
__global__ __launch_bounds__(T) void sdp_hnw2_kernel(StreamArgs a) {
  for (int b = threadIdx.x; b < a.n_inst; b += T) {
    double s0 = 0.0, s1 = 0.0;
    for (int q = 0; q < a.tile_count[b]; ++q) {
      s0 += a.tile_part[2 * (a.tile_first[b] + q)];
      s1 += a.tile_part[2 * (a.tile_first[b] + q) + 1];
    }
    const double n2 = (double)a.inst[b].n * a.inst[b].n;
    const double d0 = sqrt(s0 / n2), d1 = sqrt(s1 / n2);
    a.ctl[b].hs = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    a.ctl[b].h_try = d1;  // kept until the step size is set
  }
}

// Starting step, part 3 (tiles): yb0 = rho + hs f0.
template <int T>
__global__ __launch_bounds__(T) void sdp_hnw3_kernel(StreamArgs a) {
  const int tix = xcd_tile(a.n_tiles);
  if (tix >= a.n_tiles) return;
  const Tile tl = a.tiles[tix];
  const int64_t base = a.inst[tl.inst].rho_off;
  const double hs = a.ctl[tl.inst].hs;
  const double2 *rho = reinterpret_cast<const double2 *>(a.rho) + base;
  const double2 *K = reinterpret_cast<const double2 *>(a.K) + base;
  double2 *y = reinterpret_cast<double2 *>(a.yb0) + base;
  for (int e = tl.e0 + threadIdx.x; e < tl.e1; e += T) y[e] = caxpy(hs, K[e], rho[e]);
}

// Starting step, part 4 (tiles): f1 = L(yb0); partial sums of |(f1-f0)/sc|^2.
template <int T>
__global__ __launch_bounds__(T) void sdp_hnw4_kernel(StreamArgs a) {
  __shared__ double uq[kMaxWidth];
  __shared__ double sh[T / 64];
  const int tix = xcd_tile(a.n_tiles);
  if (tix >= a.n_tiles) return;
  const int seg0 = a.n_seg > 0 ? a.stop_seg[0] : -1;
  const TileCtx t = tile_ctx(a, tix, uq, seg0);
  __syncthreads();
  const double2 *rho = reinterpret_cast<const double2 *>(a.rho) + t.base;
  const double2 *y = reinterpret_cast<const double2 *>(a.yb0) + t.base;
  const double2 *K = reinterpret_cast<const double2 *>(a.K) + t.base;
  double p = 0.0;
  for (int e = t.e0 + threadIdx.x; e < t.e1; e += T) {
    const int i = e / t.n, j = e - i * t.n;
    const double2 f1 = lindblad_elem(t.op, y, i, j, y[e], uq);
    const double sc = a.atol + a.rtol * hypot(rho[e].x, rho[e].y);
    const double r = hypot(f1.x - K[e].x, f1.y - K[e].y) / sc;
    p += r * r;
  }
  const double tot = block_sum<T>(p, sh);
  if (threadIdx.x == 0) a.tile_part[tix] = tot;
}

// Starting step, part 5 (single workgroup): h, and the first attempt's set-up.
template <int T>
__global__ __launch_bounds__(T) void sdp_hnw5_kernel(StreamArgs a, int have_h0) {
  for (int b = threadIdx.x; b < a.n_inst; b += T) {
    DpCtl c = a.ctl[b];
    if (!have_h0) {
      double s2 = 0.0;
      for (int q = 0; q < a.tile_count[b]; ++q) s2 += a.tile_part[a.tile_first[b] + q];
      const double n2 = (double)a.inst[b].n * a.inst[b].n;
      const double hs = c.hs, d1 = c.h_try;
      const double d2 = sqrt(s2 / n2) / hs;
      const double dm = fmax(d1, d2);
      const double h1 = (dm <= 1e-15) ? fmax(1e-6, hs * 1e-3) : pow(0.01 / dm, 0.2);
      c.h = fmin(100.0 * hs, h1);
      c.k1_seg = a.n_seg > 0 ? a.stop_seg[0] : -1;
    }
    dp_setup(c, a);
    a.ctl[b] = c;
  }
}

// Counts and status of every instance (single workgroup).
template <int T>
__global__ __launch_bounds__(T) void sdp_final_kernel(StreamArgs a) {
  for (int b = threadIdx.x; b < a.n_inst; b += T) {
    if (a.counts) {
      a.counts[2 * (int64_t)b] = a.ctl[b].n_acc;
      a.counts[2 * (int64_t)b + 1] = a.ctl[b].n_rej;
    }
    if (a.status) a.status[b] = a.ctl[b].status;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int T, int EPT>
static hipError_t launch_rk4_t(const Rk4Args &a, int n_packs, int lds, hipStream_t s) {
  auto k = rk4_resident_kernel<T, EPT>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_packs), dim3(T), lds, s, a);
  return hipGetLastError();
}

}  // namespace lme

// Resident RK4 configurations: threads per workgroup x elements per thread.
extern "C" int lme_internal_rk4_configs(int *T, int *EPT, int cap) {
  static const int cfg[][2] = {{64, 1}, {64, 2}, {64, 4}, {64, 8},
                               {256, 1}, {256, 2}, {256, 4}, {256, 8}, {256, 16}, {256, 32},
                               {512, 1}, {512, 2}, {512, 4}, {512, 8}, {512, 13}, {512, 16},
                               {1024, 1}, {1024, 2}, {1024, 4}, {1024, 6}};
  const int nc = (int)(sizeof(cfg) / sizeof(cfg[0]));
  for (int i = 0; i < nc && i < cap; ++i) {
    T[i] = cfg[i][0];
    EPT[i] = cfg[i][1];
  }
  return nc;
}

extern "C" int lme_internal_blob_stride(int blob_bytes) { return lme::blob_stride_of(blob_bytes); }

extern "C" int lme_internal_pack_lds_bytes(int n, int m, int blob_bytes, int nb) {
  return lme::pack_lds_bytes(n, m, blob_bytes, nb);
}

extern "C" hipError_t lme_internal_launch_rk4(int T, int EPT, const lme::Rk4Args *a,
                                              int n_packs, int lds, hipStream_t s) {
  using namespace lme;
#define LME_RK4_CASE(TT, EE) \
  if (T == TT && EPT == EE) return launch_rk4_t<TT, EE>(*a, n_packs, lds, s);
  LME_RK4_CASE(64, 1) LME_RK4_CASE(64, 2) LME_RK4_CASE(64, 4) LME_RK4_CASE(64, 8)
  LME_RK4_CASE(256, 1) LME_RK4_CASE(256, 2) LME_RK4_CASE(256, 4) LME_RK4_CASE(256, 8)
  LME_RK4_CASE(256, 16) LME_RK4_CASE(256, 32)
  LME_RK4_CASE(512, 1) LME_RK4_CASE(512, 2) LME_RK4_CASE(512, 4) LME_RK4_CASE(512, 8)
  LME_RK4_CASE(512, 13) LME_RK4_CASE(512, 16)
  LME_RK4_CASE(1024, 1) LME_RK4_CASE(1024, 2) LME_RK4_CASE(1024, 4) LME_RK4_CASE(1024, 6)
#undef LME_RK4_CASE
  return hipErrorInvalidValue;
}

// Small instances, one element per lane (the packs of the 64 x 1 row
// configuration); the operator widths must be within the kLane* limits.
extern "C" int lme_internal_lane_fits(int wo, int nb, int wb, int nc, int wc) {
  return wo <= lme::kLaneWO && nb <= lme::kLaneNB && wb <= lme::kLaneWB &&
         nc * wc * wc <= lme::kLaneJ;
}

extern "C" hipError_t lme_internal_launch_rk4_lane(const lme::Rk4Args *a, int n_packs, int lds,
                                                   hipStream_t s) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(lme::rk4_lane_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lme::rk4_lane_kernel, dim3(n_packs), dim3(64), lds, s, *a);
  return hipGetLastError();
}

template <int T, int EPT, int WO, int NC, int NB, bool RE, bool HM>
static hipError_t launch_colown_t(const lme::Rk4Args &a, int n_packs, int lds, hipStream_t s) {
  auto k = [] {
    if constexpr (HM) return lme::rk4_herm_kernel<T, EPT, WO, NC, NB, RE>;
    else return lme::rk4_colown_kernel<T, EPT, WO, NC, NB, RE>;
  }();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_packs), dim3(T), lds, s, a);
  return hipGetLastError();
}

// Column-owner kernels: (T, EPT) configuration index cfg into kColCfg (or
// kHermCfg when herm), the operator shape (wo, nc, nb) and the
// real/imaginary specialisation re; returns hipErrorInvalidValue for shapes
// that have no instantiation.
extern "C" hipError_t lme_internal_launch_rk4_colown(int cfg, int herm, int wo, int nc, int nb,
                                                     int re, const lme::Rk4Args *a, int n_packs,
                                                     int lds, hipStream_t s) {
#define LME_COL_CASE(CFG, HM, TT, EE, W, K, B, R)                                    \
  if (cfg == CFG && herm == HM && wo == W && nc == K && nb == B && re == R)          \
    return launch_colown_t<TT, EE, W, K, B, (R != 0), (HM != 0)>(*a, n_packs, lds, s);
#define LME_COL_SHAPES(CFG, HM, TT, EE, R)                                            \
  LME_COL_CASE(CFG, HM, TT, EE, 1, 2, 0, R) LME_COL_CASE(CFG, HM, TT, EE, 1, 3, 0, R) \
  LME_COL_CASE(CFG, HM, TT, EE, 2, 2, 0, R) LME_COL_CASE(CFG, HM, TT, EE, 1, 2, 1, R) \
  LME_COL_CASE(CFG, HM, TT, EE, 1, 3, 1, R)
  LME_COL_SHAPES(0, 0, 512, 14, 0) LME_COL_SHAPES(0, 0, 512, 14, 1)
  LME_COL_SHAPES(1, 0, 768, 9, 0) LME_COL_SHAPES(1, 0, 768, 9, 1)
  LME_COL_SHAPES(0, 1, 512, 8, 0) LME_COL_SHAPES(0, 1, 512, 8, 1)
  LME_COL_SHAPES(1, 1, 768, 5, 0) LME_COL_SHAPES(1, 1, 768, 5, 1)
#undef LME_COL_SHAPES
#undef LME_COL_CASE
  return hipErrorInvalidValue;
}

extern "C" int lme_internal_colown_has_shape(int wo, int nc, int nb) {
  return (wo == 1 && nc == 2) || (wo == 1 && nc == 3) || (wo == 2 && nc == 2 && nb == 0);
}

template <int T, int EPT, int WO = 0, int NC = 0, int NB = 0, bool RE = false, bool COL = false>
static hipError_t launch_dp5_t(const lme::Dp5Args &a, int n_packs, int lds, hipStream_t s) {
  auto k = lme::dp5_resident_kernel<T, EPT, WO, NC, NB, RE, COL>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_packs), dim3(T), lds, s, a);
  return hipGetLastError();
}

// Resident Dormand-Prince: 512 threads, EPT elements per thread.
extern "C" int lme_internal_dp5_epts(int *ept, int cap) {
  static const int e[] = {1, 2, 4, 8, 16};
  for (int i = 0; i < 5 && i < cap; ++i) ept[i] = e[i];
  return 5;
}

// LDS beyond the pack proper: per-instance step control and 2 m doubles.
extern "C" int lme_internal_dp5_extra_lds(int m) {
  return lme::dp_ctl_bytes(m) + lme::align16(16 * m);
}

// Column-owner resident Dormand-Prince: 512 threads and up to EPT = 8 or 16
// rows per thread, or 1024 threads and 4 rows (EPT = 4); the column-kernel
// shapes.
extern "C" hipError_t lme_internal_launch_dp5_col(int EPT, int wo, int nc, int nb, int re,
                                                  const lme::Dp5Args *a, int n_packs, int lds,
                                                  hipStream_t s) {
#define LME_DC(E, W, K, B, R)                                                  \
  if (EPT == E && wo == W && nc == K && nb == B && re == R) {                  \
    if constexpr (E == 4)                                                      \
      return launch_dp5_t<1024, 4, W, K, B, (R != 0), true>(*a, n_packs, lds, s); \
    else                                                                       \
      return launch_dp5_t<512, E, W, K, B, (R != 0), true>(*a, n_packs, lds, s); \
  }
#define LME_DC_E(E)                                                                   \
  LME_DC(E, 1, 2, 0, 0) LME_DC(E, 1, 3, 0, 0) LME_DC(E, 2, 2, 0, 0) LME_DC(E, 1, 2, 1, 0) \
  LME_DC(E, 1, 3, 1, 0) LME_DC(E, 1, 2, 0, 1) LME_DC(E, 1, 3, 0, 1) LME_DC(E, 2, 2, 0, 1) \
  LME_DC(E, 1, 2, 1, 1) LME_DC(E, 1, 3, 1, 1)
  LME_DC_E(4) LME_DC_E(8) LME_DC_E(16)
#undef LME_DC_E
#undef LME_DC
  return hipErrorInvalidValue;
}

extern "C" hipError_t lme_internal_launch_dp5(int EPT, const lme::Dp5Args *a, int n_packs,
                                              int lds, hipStream_t s) {
  switch (EPT) {
    case 1: return launch_dp5_t<512, 1>(*a, n_packs, lds, s);
    case 2: return launch_dp5_t<512, 2>(*a, n_packs, lds, s);
    case 4: return launch_dp5_t<512, 4>(*a, n_packs, lds, s);
    case 8: return launch_dp5_t<512, 8>(*a, n_packs, lds, s);
    case 16: return launch_dp5_t<512, 16>(*a, n_packs, lds, s);
  }
  return hipErrorInvalidValue;
}

template <int T, int EPT, int NQ, int WO = 0, int NC = 0, bool COL = false>
static hipError_t launch_grad_t(const lme::GradArgs &a, int n_packs, int lds, hipStream_t s) {
  auto k = lme::grad_resident_kernel<T, EPT, NQ, WO, NC, COL>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_packs), dim3(T), lds, s, a);
  return hipGetLastError();
}

// Gradient kernel: T = 512 threads with EPT in {1, 2, 4, 8}, or T = 1024 with
// EPT in {1, 2, 4}; 1 or 2 control terms.
extern "C" hipError_t lme_internal_launch_grad(int T, int EPT, int nq, const lme::GradArgs *a,
                                               int n_packs, int lds, hipStream_t s) {
#define LME_G(TT, E, Q) \
  if (T == TT && EPT == E && nq == Q) return launch_grad_t<TT, E, Q>(*a, n_packs, lds, s);
  LME_G(512, 1, 1) LME_G(512, 2, 1) LME_G(512, 4, 1) LME_G(512, 8, 1)
  LME_G(512, 1, 2) LME_G(512, 2, 2) LME_G(512, 4, 2) LME_G(512, 8, 2)
  LME_G(1024, 1, 1) LME_G(1024, 2, 1) LME_G(1024, 4, 1)
  LME_G(1024, 1, 2) LME_G(1024, 2, 2) LME_G(1024, 4, 2)
#undef LME_G
  return hipErrorInvalidValue;
}

// Column-owner gradient kernel: T threads, EPT rows per thread, one control
// term, real structure, operator shape (wo, nc) of the column kernels.
extern "C" hipError_t lme_internal_launch_grad_col(int T, int EPT, int wo, int nc,
                                                   const lme::GradArgs *a, int n_packs, int lds,
                                                   hipStream_t s) {
#define LME_GC(TT, E, W, K)                           \
  if (T == TT && EPT == E && wo == W && nc == K)      \
    return launch_grad_t<TT, E, 1, W, K, true>(*a, n_packs, lds, s);
  LME_GC(512, 4, 1, 2) LME_GC(512, 4, 1, 3)
#undef LME_GC
  return hipErrorInvalidValue;
}

extern "C" hipError_t lme_internal_launch_apply_global(const lme::ApplyGArgs *a, hipStream_t s) {
  const int grid = 8 * ((a->n_tiles + 7) / 8);
  hipLaunchKernelGGL(lme::apply_global_kernel<256>, dim3(grid), dim3(256), 0, s, *a);
  return hipGetLastError();
}

// Row-block streamed application: R = 16 rows per tile (n <= 256) or 4
// (n <= 1024); lds = R * max n * 16 bytes.
extern "C" hipError_t lme_internal_launch_apply_rows(int R, int re, const lme::ApplyGArgs *a,
                                                    int lds, hipStream_t s) {
  const int grid = 8 * ((a->n_tiles + 7) / 8);
  auto go = [&](auto k) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(R == 16 ? 256 * 16 / lme::kRowsRT : 256), lds, s, *a);
    return hipGetLastError();
  };
  if (R == 16)
    return re ? go(lme::apply_rows_kernel<16, lme::kRowsRT, true>)
              : go(lme::apply_rows_kernel<16, lme::kRowsRT, false>);
  if (R == 4) return re ? go(lme::apply_rows_kernel<4, 4, true>) : go(lme::apply_rows_kernel<4, 4, false>);
  return hipErrorInvalidValue;
}

extern "C" hipError_t lme_internal_launch_superop(const lme::SuperArgs *a, hipStream_t s) {
  const int grid = 8 * ((a->n_tiles + 7) / 8);
  hipLaunchKernelGGL(lme::superop_kernel<256>, dim3(grid), dim3(256), 0, s, *a);
  return hipGetLastError();
}

template <int WO, int NC, int NB, bool RE>
static hipError_t launch_apply_shape_t(const lme::ApplyArgs &a, int n_packs, int lds,
                                       hipStream_t s) {
  auto k = lme::apply_shape_kernel<1024, WO, NC, NB, RE>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_packs), dim3(1024), lds, s, a);
  return hipGetLastError();
}

template <int T, int WO, int NC, int NB, bool RE>
static hipError_t launch_apply_col_t(const lme::ApplyArgs &a, int n_packs, int lds,
                                     hipStream_t s) {
  auto k = lme::apply_col_kernel<T, WO, NC, NB, RE>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_packs), dim3(T), lds, s, a);
  return hipGetLastError();
}

// Column-owner application, T in {256, 512, 1024} threads (the column-kernel
// shapes).
extern "C" hipError_t lme_internal_launch_apply_col(int T, int wo, int nc, int nb, int re,
                                                    const lme::ApplyArgs *a, int n_packs,
                                                    int lds, hipStream_t s) {
#define LME_AC(TT, W, K, B, R) \
  if (T == TT && wo == W && nc == K && nb == B && re == R) \
    return launch_apply_col_t<TT, W, K, B, (R != 0)>(*a, n_packs, lds, s);
#define LME_AC_T(TT)                                                                     \
  LME_AC(TT, 1, 2, 0, 0) LME_AC(TT, 1, 3, 0, 0) LME_AC(TT, 2, 2, 0, 0)                   \
  LME_AC(TT, 1, 2, 1, 0) LME_AC(TT, 1, 3, 1, 0) LME_AC(TT, 1, 2, 0, 1)                   \
  LME_AC(TT, 1, 3, 0, 1) LME_AC(TT, 2, 2, 0, 1) LME_AC(TT, 1, 2, 1, 1) LME_AC(TT, 1, 3, 1, 1)
  LME_AC_T(256) LME_AC_T(512) LME_AC_T(1024)
#undef LME_AC_T
#undef LME_AC
  return hipErrorInvalidValue;
}

template <int WO, int NC, int NB, bool RE>
static hipError_t launch_apply_pipe_t(const lme::PipeArgs &a, int grid, hipStream_t s) {
  auto k = lme::apply_pipe_kernel<WO, NC, NB, RE>;
  const int lds = 2 * lme::kPipeStage + lme::kPipeMaxTiles * (int)sizeof(lme::PTile) + 16;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid), dim3(lme::kPipeT), lds, s, a);
  return hipGetLastError();
}

// Pipelined column application (the column-kernel shapes).
extern "C" hipError_t lme_internal_launch_apply_pipe(int wo, int nc, int nb, int re,
                                                     const lme::PipeArgs *a, int grid,
                                                     hipStream_t s) {
#define LME_AP(W, K, B, R) \
  if (wo == W && nc == K && nb == B && re == R) \
    return launch_apply_pipe_t<W, K, B, (R != 0)>(*a, grid, s);
  LME_AP(1, 2, 0, 0) LME_AP(1, 3, 0, 0) LME_AP(2, 2, 0, 0) LME_AP(1, 2, 1, 0) LME_AP(1, 3, 1, 0)
  LME_AP(1, 2, 0, 1) LME_AP(1, 3, 0, 1) LME_AP(2, 2, 0, 1) LME_AP(1, 2, 1, 1) LME_AP(1, 3, 1, 1)
#undef LME_AP
  return hipErrorInvalidValue;
}

// Shape-specialised application (the shapes of the column-owner kernels).
extern "C" hipError_t lme_internal_launch_apply_shape(int wo, int nc, int nb, int re,
                                                      const lme::ApplyArgs *a, int n_packs,
                                                      int lds, hipStream_t s) {
#define LME_AS(W, K, B, R) \
  if (wo == W && nc == K && nb == B && re == R) \
    return launch_apply_shape_t<W, K, B, (R != 0)>(*a, n_packs, lds, s);
  LME_AS(1, 2, 0, 0) LME_AS(1, 3, 0, 0) LME_AS(2, 2, 0, 0) LME_AS(1, 2, 1, 0) LME_AS(1, 3, 1, 0)
  LME_AS(1, 2, 0, 1) LME_AS(1, 3, 0, 1) LME_AS(2, 2, 0, 1) LME_AS(1, 2, 1, 1) LME_AS(1, 3, 1, 1)
#undef LME_AS
  return hipErrorInvalidValue;
}

// Streamed steppers: kernel `which` of the sequences (see the host).
extern "C" hipError_t lme_internal_launch_sdp(int which, int arg, const lme::StreamArgs *a,
                                              hipStream_t s) {
  using namespace lme;
  const int grid = 8 * ((a->n_tiles + 7) / 8);
  switch (which) {
    case 0: hipLaunchKernelGGL(sdp_stage_kernel<256>, dim3(grid), dim3(256), 0, s, *a, arg); break;
    case 1: hipLaunchKernelGGL(sdp_control_kernel<1024>, dim3(1), dim3(1024), 0, s, *a); break;
    case 2: hipLaunchKernelGGL(sdp_accept_kernel<256>, dim3(grid), dim3(256), 0, s, *a); break;
    case 3: hipLaunchKernelGGL(stream_output_kernel<256>, dim3(a->n_inst), dim3(256), 0, s, *a, arg); break;
    case 4: hipLaunchKernelGGL(sdp_init_kernel<1024>, dim3(1), dim3(1024), 0, s, *a); break;
    case 5: hipLaunchKernelGGL(sdp_hnw1_kernel<256>, dim3(grid), dim3(256), 0, s, *a); break;
    case 6: hipLaunchKernelGGL(sdp_hnw2_kernel<1024>, dim3(1), dim3(1024), 0, s, *a); break;
    case 7: hipLaunchKernelGGL(sdp_hnw3_kernel<256>, dim3(grid), dim3(256), 0, s, *a); break;
    case 8: hipLaunchKernelGGL(sdp_hnw4_kernel<256>, dim3(grid), dim3(256), 0, s, *a); break;
    case 9: hipLaunchKernelGGL(sdp_hnw5_kernel<1024>, dim3(1), dim3(1024), 0, s, *a, arg); break;
    case 10: hipLaunchKernelGGL(sdp_final_kernel<1024>, dim3(1), dim3(1024), 0, s, *a); break;
    case 20: hipLaunchKernelGGL(srk_stage_kernel<256>, dim3(grid), dim3(256), 0, s, *a, arg); break;
    case 21: hipLaunchKernelGGL(srk_output_kernel<256>, dim3(a->n_inst), dim3(256), 0, s, *a); break;
    case 22: hipLaunchKernelGGL(srk_tail_kernel, dim3(1), dim3(1), 0, s, *a, arg); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Row-block stage kernel of the streamed adaptive stepper (16-row tiles):
// prepare sets its dynamic LDS limit (outside any graph capture), launch
// issues stage s.
template <bool RE>
static auto sdp_rows_kernel() {
  return lme::sdp_stage_rows_kernel<16, lme::kRowsRT, RE>;
}
extern "C" hipError_t lme_internal_sdp_rows_prepare(int re, int lds) {
  const void *k = re ? reinterpret_cast<const void *>(sdp_rows_kernel<true>())
                     : reinterpret_cast<const void *>(sdp_rows_kernel<false>());
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}
extern "C" hipError_t lme_internal_launch_sdp_rows(int s, int re, const lme::StreamArgs *a,
                                                   int lds, hipStream_t st) {
  const int grid = 8 * ((a->n_tiles + 7) / 8);
  const dim3 block(256 * 16 / lme::kRowsRT);
  if (re)
    hipLaunchKernelGGL(sdp_rows_kernel<true>(), dim3(grid), block, lds, st, *a, s);
  else
    hipLaunchKernelGGL(sdp_rows_kernel<false>(), dim3(grid), block, lds, st, *a, s);
  return hipGetLastError();
}

extern "C" hipError_t lme_internal_launch_apply_lds(const lme::ApplyArgs *a, int n_packs,
                                                    int lds, hipStream_t s) {
  auto k = lme::apply_lds_kernel<1024>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_packs), dim3(1024), lds, s, *a);
  return hipGetLastError();
}
