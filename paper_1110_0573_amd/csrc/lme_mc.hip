// lme_mc.hip -- Monte-Carlo wave-function trajectories on gfx950.
//
// What is computed (arXiv:1110.0573, Sec. 3.2, steps I-IV): every trajectory
// evolves a ket under the effective Hamiltonian of Eq. (heff),
//   d psi/dt = A psi,   A = -i H_eff = -i H - 1/2 sum_n C_n^+ C_n,
// until its squared norm falls to the drawn number r (step II), then jumps
// with the collapse operator chosen by the cumulative rule of Eq. (mc3) with
// a second draw r' (Eq. (pcn) gives the probabilities), is renormalised
// (Eq. (project)) and continues with the next draw (step IV).
//
// Integrator: classic RK4 on the grid t0 + m h.  For the autonomous linear
// equation the RK4 step of length s is exactly the degree-4 Taylor polynomial
//   psi(s) = v0 + s v1 + s^2 v2 + s^3 v3 + s^4 v4,  v0 = psi, v_k = A v_{k-1} / k,
// which is how it is evaluated here: the v_k do not depend on s, so
//   * every trajectory of a workgroup can take its own step length (the rest
//     of a grid step after a jump) in one uniform pass, and
//   * the jump time is a root of the scalar polynomial |psi(s)|^2 - r, whose
//     nine coefficients c_d = sum_{j+k=d} Re <v_j|v_k> come from one
//     reduction; bisection on that polynomial replaces repeated integration.
//
// Work decomposition: a workgroup holds P trajectories; G = 2^g threads own
// one trajectory, thread g its rows g, g + G, ... (R rows).  The current
// Taylor vector of every trajectory is staged in LDS (16 n bytes each) so the
// sparse products gather from LDS; the state psi sits in LDS too (read and
// written only by the thread that owns the row) and the running sum in
// registers.  Per-trajectory scalars (threshold, time left, jump count,
// status) are identical in every thread of a group: reductions end with the
// same bits in every lane (xor butterflies, then a fixed-order sum of the
// wave partials), so every decision is taken uniformly without broadcasts.
// Workgroups are persistent and walk the packs of P trajectories.
#include <hip/hip_runtime.h>

#include "../../include/lme.h"
#include "lme_internal.h"

namespace {

using lme::McArgs;

struct __attribute__((aligned(16))) cplx {
  double x, y;
};

__device__ inline cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline cplx cfma(cplx a, cplx b, cplx c) {  // a * b + c
  return {fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}
__device__ inline cplx cscale(double s, cplx a) { return {s * a.x, s * a.y}; }
__device__ inline cplx caxpy(double s, cplx a, cplx c) { return {fma(s, a.x, c.x), fma(s, a.y, c.y)}; }
__device__ inline double cabs2(cplx a) { return fma(a.x, a.x, a.y * a.y); }
// An opaque copy: the compiler cannot prove it equal to its input.
__device__ inline int launder(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Sum of NV values over the G threads of each trajectory group.  Every
// thread of the group gets bitwise the same sums.  red: LDS, NV doubles per
// wave.  Must be called by every thread of the workgroup (it may contain
// barriers).
template <int NV>
__device__ inline void group_sum(double (&v)[NV], int G, double *red) {
  const int lane = threadIdx.x & 63;
  if (G <= 64) {
    for (int off = G >> 1; off > 0; off >>= 1)
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] += __shfl_xor(v[q], off, 64);
    return;
  }
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] += __shfl_xor(v[q], off, 64);
  const int wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[wave * NV + q] = v[q];
  __syncthreads();
  const int wpg = G >> 6;                      // waves per group
  const int w0 = (threadIdx.x / G) * wpg;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = red[w0 * NV + q];
    for (int w = 1; w < wpg; ++w) s += red[(w0 + w) * NV + q];
    v[q] = s;
  }
  __syncthreads();
}

// Operator tables read through buffer resources (base and size in scalar
// registers, a 32-bit byte offset per lane): no 64-bit address per row stays
// live across the step loop.
constexpr int kBufferFlags = 0x00020000;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct Tabs {
  __amdgpu_buffer_rsrc_t D, Oval, Ocol, Jval, Jcol, Eval, Ecol, vb;
};

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void *p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, kBufferFlags);
}
__device__ inline cplx ld_c(__amdgpu_buffer_rsrc_t r, uint32_t idx) {
  return __builtin_bit_cast(cplx, __builtin_amdgcn_raw_buffer_load_b128(r, idx * 16u, 0, 0));
}
__device__ inline int ld_i(__amdgpu_buffer_rsrc_t r, uint32_t idx) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(r, idx * 4u, 0, 0);
}
__device__ inline void st_c(__amdgpu_buffer_rsrc_t r, uint32_t idx, cplx v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, idx * 16u, 0, 0);
}

// y = (A x)_i for row i, x = the group's vector in LDS.
__device__ inline cplx row_apply(const Tabs &t, int n, int wo, const cplx *x, int i) {
  cplx acc = cmul(ld_c(t.D, i), x[i]);
  for (int s = 0; s < wo; ++s) acc = cfma(ld_c(t.Oval, s * n + i), x[ld_i(t.Ocol, s * n + i)], acc);
  return acc;
}

// (C_k x)_i
__device__ inline cplx row_jump(const Tabs &t, int n, int wc, const cplx *x, int k, int i) {
  cplx acc = {0.0, 0.0};
  const int base = k * wc * n;
  for (int s = 0; s < wc; ++s)
    acc = cfma(ld_c(t.Jval, base + s * n + i), x[ld_i(t.Jcol, base + s * n + i)], acc);
  return acc;
}

// (E_m x)_i
__device__ inline cplx row_eop(const Tabs &t, int n, int we, const cplx *x, int m, int i) {
  cplx acc = {0.0, 0.0};
  const int base = m * we * n;
  for (int s = 0; s < we; ++s)
    acc = cfma(ld_c(t.Eval, base + s * n + i), x[ld_i(t.Ecol, base + s * n + i)], acc);
  return acc;
}

constexpr int kMaxNC = lme::kMcMaxNC;

// Largest workgroup of the kernel with R rows per thread.
constexpr int mc_max_threads(int) { return 512; }

template <int R>
__global__ __launch_bounds__(mc_max_threads(R)) void mc_kernel(McArgs a) {
  extern __shared__ double lds[];
  const int G = a.G, P = a.P, n = a.n;
  const int nwaves = (blockDim.x + 63) >> 6;
  double *red = lds;                                     // [nwaves][9] wave partials
  double *wts = lds + nwaves * 9;                        // [P][kMaxNC] jump weights
  cplx *V = reinterpret_cast<cplx *>(lds + ((nwaves * 9 + P * kMaxNC + 1) & ~1));
  const int p = threadIdx.x / G;                         // trajectory slot
  const int g0 = threadIdx.x % G;
  cplx *X = V + (size_t)p * n;                           // this group's Taylor vector
  cplx *PS = V + (size_t)(P + p) * n;                    // this group's state psi
  const bool in_group = p < P;
  const cplx *psi0 = reinterpret_cast<const cplx *>(a.psi0);
  cplx *ex = reinterpret_cast<cplx *>(a.ex_traj);
  const int n_packs = (a.n_traj + P - 1) / P;
  const int64_t dstride = 2LL * (a.max_jumps + 1);
  Tabs tb;
  tb.D = rsrc(a.D, 16LL * n);
  tb.Oval = rsrc(a.Oval, 16LL * a.wo * n);
  tb.Ocol = rsrc(a.Ocol, 4LL * a.wo * n);
  tb.Jval = rsrc(a.Jval, 16LL * a.nc * a.wc * n);
  tb.Jcol = rsrc(a.Jcol, 4LL * a.nc * a.wc * n);
  tb.Eval = rsrc(a.Eval, 16LL * a.ne * a.we * n);
  tb.Ecol = rsrc(a.Ecol, 4LL * a.ne * a.we * n);
  tb.vb = rsrc(a.vbuf + (size_t)blockIdx.x * 8 * P * n, 64LL * P * n);

  for (int pack = blockIdx.x; pack < n_packs; pack += gridDim.x) {
    // g is re-read here, in every sub-step, output and jump (opaque copies),
    // so the row indices and offsets derived from it are recomputed where
    // they are used instead of being hoisted out of the loops and spilled
    int g = launder(g0);
    const int traj = pack * P + p;
    const bool alive0 = in_group && traj < a.n_traj;
    // the initial ket, normalised, into PS (each thread its own rows)
    double nn[1] = {0.0};
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = g + q * G;
      if (alive0 && i < n) nn[0] += cabs2(psi0[i]);
    }
    group_sum<1>(nn, G, red);
    const double sc = nn[0] > 0.0 ? 1.0 / sqrt(nn[0]) : 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = g + q * G;
      if (in_group && i < n) PS[i] = alive0 ? cscale(sc, psi0[i]) : cplx{0.0, 0.0};
    }
    // outputs of a trajectory that stops early stay zero
    if (alive0)
      for (int e = g; e < a.ne * a.n_t; e += G) ex[(size_t)traj * a.ne * a.n_t + e] = {0.0, 0.0};
    int status = (alive0 && !(nn[0] > 0.0 && isfinite(nn[0]))) ? LME_EINVAL : LME_OK;
    bool alive = alive0 && status == LME_OK;
    int jumps = 0;
    const double *dr = a.draws + (alive0 ? traj * dstride : 0);
    double r = alive ? dr[0] : 0.0;
    int next_out = 0;

    // <psi|E_m|psi> / <psi|psi> of every trajectory at output k (operators
    // reduced two at a time)
    auto record = [&](int k) {
      g = launder(g0);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = g + q * G;
        if (in_group && i < n) X[i] = PS[i];
      }
      __syncthreads();
      for (int m0 = 0; m0 < a.ne; m0 += 2) {
        double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = g + q * G;
          if (in_group && i < n) {
            const cplx ps = X[i];
#pragma unroll
            for (int d = 0; d < 2; ++d)
              if (m0 + d < a.ne) {
                const cplx e = row_eop(tb, n, a.we, X, m0 + d, i);
                // conj(psi_i) * (E psi)_i
                v[2 * d] += ps.x * e.x + ps.y * e.y;
                v[2 * d + 1] += ps.x * e.y - ps.y * e.x;
              }
            v[4] += cabs2(ps);
          }
        }
        group_sum<5>(v, G, red);
        if (alive && g == 0)
#pragma unroll
          for (int d = 0; d < 2; ++d)
            if (m0 + d < a.ne)
              ex[((size_t)traj * a.ne + m0 + d) * a.n_t + k] = {v[2 * d] / v[4], v[2 * d + 1] / v[4]};
      }
    };

    for (int st = 0; st <= a.nsteps; ++st) {
      // outputs due at grid point st (output 0 at the initial time)
      while (next_out < a.n_t && (next_out == 0 || a.out_step[next_out] == st)) record(next_out++);
      if (st == a.nsteps) break;
      double t = a.t0 + (double)st * a.h;   // time of the current state
      double left = alive ? a.h : 0.0;      // rest of this grid step
      for (;;) {
        if (!__syncthreads_or(left > 0.0)) break;
        g = launder(g0);
        const double s = left;
        cplx acc[R];
        // Taylor form of the RK4 step of length s: acc = sum_k s^k v_k
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = g + q * G;
          acc[q] = (in_group && i < n) ? PS[i] : cplx{0.0, 0.0};
          if (in_group && i < n) X[i] = acc[q];
        }
        double sk = 1.0;
        for (int k = 1; k <= 4; ++k) {
          __syncthreads();
          cplx y[R];
          const double inv = 1.0 / (double)k;
          sk *= s;
#pragma unroll
          for (int q = 0; q < R; ++q) {
            const int i = g + q * G;
            y[q] = (in_group && i < n) ? cscale(inv, row_apply(tb, n, a.wo, X, i)) : cplx{0.0, 0.0};
            acc[q] = caxpy(sk, y[q], acc[q]);
          }
          if (k < 4) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < R; ++q) {
              const int i = g + q * G;
              if (in_group && i < n) X[i] = y[q];
            }
          }
        }
        double nt[1] = {0.0};
#pragma unroll
        for (int q = 0; q < R; ++q) nt[0] += cabs2(acc[q]);
        group_sum<1>(nt, G, red);
        bool cross = false;
        if (left > 0.0) {
          if (!isfinite(nt[0])) {
            status = LME_ENONFINITE;
            alive = false;
            left = 0.0;
          } else if (nt[0] > r) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
              const int i = g + q * G;
              if (in_group && i < n) PS[i] = acc[q];
            }
            left = 0.0;
          } else {
            cross = true;
          }
        }
        if (!__syncthreads_or(cross)) continue;
        g = launder(g0);

        // ---- a jump inside this sub-step for at least one trajectory ----
        // recompute v1..v4 from psi (unchanged for the crossing ones), keep
        // them in this workgroup's slice of the scratch buffer
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = g + q * G;
          if (in_group && i < n) X[i] = PS[i];
        }
        for (int k = 1; k <= 4; ++k) {
          __syncthreads();
          cplx y[R];
          const double inv = 1.0 / (double)k;
#pragma unroll
          for (int q = 0; q < R; ++q) {
            const int i = g + q * G;
            y[q] = (in_group && i < n) ? cscale(inv, row_apply(tb, n, a.wo, X, i)) : cplx{0.0, 0.0};
            if (in_group && i < n) st_c(tb.vb, ((k - 1) * P + p) * n + i, y[q]);
          }
          __syncthreads();
#pragma unroll
          for (int q = 0; q < R; ++q) {
            const int i = g + q * G;
            if (in_group && i < n) X[i] = y[q];
          }
        }
        // coefficients of |psi(x)|^2 = sum_d c_d x^d
        double c[9];
#pragma unroll
        for (int d = 0; d < 9; ++d) c[d] = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = g + q * G;
          if (in_group && i < n) {
            cplx v[5];
            v[0] = PS[i];
#pragma unroll
            for (int k = 1; k <= 4; ++k) v[k] = ld_c(tb.vb, ((k - 1) * P + p) * n + i);
#pragma unroll
            for (int j = 0; j <= 4; ++j) {
              c[2 * j] += cabs2(v[j]);
#pragma unroll
              for (int k = j + 1; k <= 4; ++k)
                c[j + k] += 2.0 * (v[j].x * v[k].x + v[j].y * v[k].y);
            }
          }
        }
        group_sum<9>(c, G, red);
        double tau = 0.0;
        if (cross) {
          // bisection on (0, left]: the norm is above r at 0, at most r at left
          double lo = 0.0, hi = left;
          for (int it = 0; it < 400; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (!(mid > lo && mid < hi)) break;
            double pv = c[8];
            for (int d = 7; d >= 0; --d) pv = fma(pv, mid, c[d]);
            if (pv <= r)
              hi = mid;
            else
              lo = mid;
          }
          tau = hi;
        }
        __syncthreads();
        // psi(tau) by Horner into X (crossing trajectories)
        if (cross)
#pragma unroll
          for (int q = 0; q < R; ++q) {
            const int i = g + q * G;
            if (in_group && i < n) {
              cplx h4 = ld_c(tb.vb, (3 * P + p) * n + i);
              for (int k = 3; k >= 1; --k) {
                const cplx vk = ld_c(tb.vb, ((k - 1) * P + p) * n + i);
                h4 = {fma(h4.x, tau, vk.x), fma(h4.y, tau, vk.y)};
              }
              const cplx v0 = PS[i];
              X[i] = {fma(h4.x, tau, v0.x), fma(h4.y, tau, v0.y)};
            }
          }
        __syncthreads();
        // jump weights <psi|C_k^+ C_k|psi> at tau, four operators at a time,
        // into this trajectory's slots of wts
        for (int k0 = 0; k0 < a.nc; k0 += 4) {
          double w4[4] = {0.0, 0.0, 0.0, 0.0};
          if (cross)
#pragma unroll
            for (int q = 0; q < R; ++q) {
              const int i = g + q * G;
              if (in_group && i < n)
#pragma unroll
                for (int d = 0; d < 4; ++d)
                  if (k0 + d < a.nc) w4[d] += cabs2(row_jump(tb, n, a.wc, X, k0 + d, i));
            }
          group_sum<4>(w4, G, red);
          if (g == 0)
#pragma unroll
            for (int d = 0; d < 4; ++d)
              if (k0 + d < a.nc) wts[p * kMaxNC + k0 + d] = w4[d];
        }
        __syncthreads();
        if (cross) {
          if (jumps >= a.max_jumps) {
            status = LME_EDRAWS;
            alive = false;
            left = 0.0;
          } else {
            const double r2 = dr[2 * jumps + 1];
            const double *w = wts + p * kMaxNC;
            double total = 0.0;
            for (int k = 0; k < a.nc; ++k) total += w[k];
            if (!(total > 0.0) || !isfinite(total)) {
              status = LME_ENONFINITE;
              alive = false;
              left = 0.0;
            } else {
              int chosen = -1, last_nonzero = -1;
              double cum = 0.0, w_chosen = 0.0, w_last = 0.0;
              for (int k = 0; k < a.nc; ++k)
                if (chosen < 0) {
                  if (w[k] > 0.0) {
                    last_nonzero = k;
                    w_last = w[k];
                  }
                  cum += w[k] / total;
                  if (cum >= r2 && w[k] > 0.0) {
                    chosen = k;
                    w_chosen = w[k];
                  }
                }
              if (chosen < 0) {
                chosen = last_nonzero;
                w_chosen = w_last;
              }
              // the projected, renormalised state (Eq. (project)) into PS
              const double rs = 1.0 / sqrt(w_chosen);
#pragma unroll
              for (int q = 0; q < R; ++q) {
                const int i = g + q * G;
                if (in_group && i < n) PS[i] = cscale(rs, row_jump(tb, n, a.wc, X, chosen, i));
              }
              t += tau;
              if (g == 0) {
                if (a.jump_t) a.jump_t[(size_t)traj * a.max_jumps + jumps] = t;
                if (a.jump_op) a.jump_op[(size_t)traj * a.max_jumps + jumps] = chosen;
              }
              ++jumps;
              r = dr[2 * jumps];
              left -= tau;
            }
          }
        }
      }
    }
    if (alive0 && g == 0) {
      if (a.n_jumps) a.n_jumps[traj] = jumps;
      if (a.status) a.status[traj] = status;
    }
    __syncthreads();   // PS and X are reused by the next pack
  }
}

// expect[m][k] = (sum over trajectories, in order, of ex_traj[b][m][k]) / n_traj
__global__ void mc_average_kernel(const double *ex_traj, double *expect, int n_traj, int per) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per) return;
  double sx = 0.0, sy = 0.0;
  for (int b = 0; b < n_traj; ++b) {
    sx += ex_traj[2 * ((size_t)b * per + e)];
    sy += ex_traj[2 * ((size_t)b * per + e) + 1];
  }
  expect[2 * e] = sx / (double)n_traj;
  expect[2 * e + 1] = sy / (double)n_traj;
}

template <int R>
hipError_t launch_r(const McArgs *a, int grid, int lds, hipStream_t s) {
  auto k = mc_kernel<R>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid), dim3(a->P * a->G), lds, s, *a);
  return hipGetLastError();
}

}  // namespace

// Rows per thread the Monte-Carlo kernel is compiled for (ascending) and the
// largest workgroup of each.
extern "C" int lme_internal_mc_rows(int *rows, int *max_threads, int cap) {
  static const int kR[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
  const int nr = (int)(sizeof kR / sizeof kR[0]);
  for (int i = 0; i < nr && i < cap; ++i) {
    rows[i] = kR[i];
    max_threads[i] = mc_max_threads(kR[i]);
  }
  return nr;
}

// Dynamic LDS of a workgroup of T threads holding P vectors of dimension n.
extern "C" int lme_internal_mc_lds_bytes(int T, int P, int n) {
  const int nwaves = (T + 63) / 64;
  return 8 * ((nwaves * 9 + P * kMaxNC + 1) & ~1) + 32 * P * n;   // + X and psi
}

extern "C" hipError_t lme_internal_launch_mc(int R, const McArgs *a, int grid, int lds,
                                             hipStream_t s) {
  switch (R) {
    case 1: return launch_r<1>(a, grid, lds, s);
    case 2: return launch_r<2>(a, grid, lds, s);
    case 3: return launch_r<3>(a, grid, lds, s);
    case 4: return launch_r<4>(a, grid, lds, s);
    case 5: return launch_r<5>(a, grid, lds, s);
    case 6: return launch_r<6>(a, grid, lds, s);
    case 8: return launch_r<8>(a, grid, lds, s);
    case 10: return launch_r<10>(a, grid, lds, s);
    case 12: return launch_r<12>(a, grid, lds, s);
    case 16: return launch_r<16>(a, grid, lds, s);
    default: return hipErrorInvalidValue;
  }
}

extern "C" hipError_t lme_internal_launch_mc_average(const double *ex_traj, double *expect,
                                                     int n_traj, int per, hipStream_t s) {
  const int T = 256;
  hipLaunchKernelGGL(mc_average_kernel, dim3((per + T - 1) / T), dim3(T), 0, s, ex_traj, expect,
                     n_traj, per);
  return hipGetLastError();
}
