// lme_prop.hip -- propagators and the steady state of repeated propagation.
//
// The propagator U of an instance (dimension n) is the n^2 x n^2 matrix
// with vec(rho(t1)) = U vec(rho(t0)) (row-major vec), column c = vec of the
// solution from |i><j|, c = i n + j, stored column-major.  It is integrated
// as a batch of n^2 Hermitian basis matrices (so the Hermitian kernels,
// which compute each pair {i, j} once, apply) and recombined.  The steady state of repeated
// application is the limit of U^(2^k): the columns converge to Tr(X) rho_ss.
// Squaring is a dense complex FP64 matrix product on the matrix cores
// (v_mfma_f64_16x16x4f64): a 64 x 64 output tile per workgroup, panels
// staged through LDS, the real and imaginary parts as four real products per
// k-step.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

namespace {

typedef double double4v __attribute__((ext_vector_type(4)));

// Hermitian basis of the n^2 x n^2 block, column c = a n + b: |a><a| for
// a = b; X = |a><b| + |b><a| for a < b; Y = i(|b><a| - |a><b|) for a > b
// (the pair's second Hermitian combination).  Evolved with the Hermitian
// kernels, the columns give U|p><q| = (U X - i U Y) / 2 and U|q><p| =
// (U X + i U Y) / 2 (prop_combine_kernel).  Column-major blocks at off4[b].
__global__ void prop_hbasis_kernel(double *U, const int64_t *off4, const int32_t *dims,
                                   int n_inst) {
  const int b = blockIdx.y;
  if (b >= n_inst) return;
  const int n = dims[b];
  const int64_t N = (int64_t)n * n;
  double2 *Ub = reinterpret_cast<double2 *>(U) + off4[b];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N * N;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / N, r = e - c * N;
    const int ca = (int)(c / n), cb = (int)(c - (int64_t)ca * n);   // column c = |ca><cb|'s slot
    const int ra = (int)(r / n), rb = (int)(r - (int64_t)ra * n);   // element (ra, rb)
    double2 v = make_double2(0.0, 0.0);
    if (ca == cb) {
      if (ra == ca && rb == cb) v.x = 1.0;
    } else if (ca < cb) {
      if ((ra == ca && rb == cb) || (ra == cb && rb == ca)) v.x = 1.0;
    } else {   // Y for the pair (cb, ca): i |cb><ca| - i |ca><cb|
      if (ra == cb && rb == ca) v.y = 1.0;
      if (ra == ca && rb == cb) v.y = -1.0;
    }
    Ub[e] = v;
  }
}

// From the evolved Hermitian basis to the |i><j| basis, in place: for every
// pair a < b the columns c = a n + b (X) and c' = b n + a (Y) become
// (X - i Y) / 2 and (X + i Y) / 2.  Grid (blocks, n_inst); the thread of
// element (row r, column c) with c = a n + b, a < b, updates both columns.
__global__ void prop_combine_kernel(double *U, const int64_t *off4, const int32_t *dims,
                                    int n_inst) {
  const int b = blockIdx.y;
  if (b >= n_inst) return;
  const int n = dims[b];
  const int64_t N = (int64_t)n * n;
  double2 *Ub = reinterpret_cast<double2 *>(U) + off4[b];
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < N * N;
       w += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = w / N, r = w - c * N;
    const int ca = (int)(c / n), cb = (int)(c - (int64_t)ca * n);
    if (ca >= cb) continue;
    double2 *X = Ub + c * N, *Y = Ub + ((int64_t)cb * n + ca) * N;
    const double2 x = X[r], y = Y[r];
    // -i y = (y.y, -y.x); +i y = (-y.y, y.x)
    X[r] = make_double2(0.5 * (x.x + y.y), 0.5 * (x.y - y.x));
    Y[r] = make_double2(0.5 * (x.x - y.y), 0.5 * (x.y + y.x));
  }
}

// C = A B for one instance, one 64 x 64 output tile per workgroup of four
// wavefronts (each a 32 x 32 quarter: 2 x 2 matrix-core tiles of 16 x 16).
// Tiles of instance b: (N/64 rounded up)^2, listed in tiles[] as (b, ti, tj).
// The k dimension advances 16 at a time through LDS (32 measured slower:
// half the workgroups per CU for its 66 KB of panels): A's 64 x 16 panel and
// B's 16 x 64 panel (both stored k-major, B's rows padded by one element so
// that its transposing store spreads over the banks; padding A's rows as
// well measured no faster).
struct GemmTile {
  int32_t b, ti, tj, pad;
};

constexpr int kGemmTile = 64, kGemmK = 16;

// Lane layout of v_mfma_f64_16x16x4f64 (wave64): A[i][k] in lane i + 16 k,
// B[k][j] in lane j + 16 k; the four accumulator elements q of lane
// j + 16 g hold D[4 q + g][j] (rows interleaved by lane group, measured).
__global__ __launch_bounds__(256) void zgemm_kernel(const GemmTile *tiles, int n_tiles,
                                                    const int64_t *off4, const int32_t *dims,
                                                    const double *A, const double *B, double *C) {
  __shared__ double2 As[kGemmK][kGemmTile];
  __shared__ double2 Bs[kGemmK][kGemmTile + 1];
  const int t = blockIdx.x;
  if (t >= n_tiles) return;
  const GemmTile tl = tiles[t];
  const int N = dims[tl.b] * dims[tl.b];
  const int64_t o = off4[tl.b];
  const double2 *Ab = reinterpret_cast<const double2 *>(A) + o;
  const double2 *Bb = reinterpret_cast<const double2 *>(B) + o;
  double2 *Cb = reinterpret_cast<double2 *>(C) + o;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = tl.ti * kGemmTile, c0 = tl.tj * kGemmTile;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  double4v re[2][2], im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      re[a][b] = double4v{0, 0, 0, 0};
      im[a][b] = double4v{0, 0, 0, 0};
    }
  // the next panels are loaded into registers while the current ones are
  // multiplied, then stored to LDS
  double2 pa[4], pb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      // A panel: column k0 + ka, rows r0 .. r0 + 63 (contiguous in A)
      const int ka = idx >> 6, ra = idx & 63;
      const int row = r0 + ra, kk = k0 + ka;
      pa[q] = (row < N && kk < N) ? Ab[(int64_t)kk * N + row] : double2{0.0, 0.0};
      // B panel: column c0 + cb, rows k0 .. k0 + 15 (contiguous in B)
      const int cb = idx >> 4, kb = idx & 15;
      const int col = c0 + cb, kr = k0 + kb;
      pb[q] = (col < N && kr < N) ? Bb[(int64_t)col * N + kr] : double2{0.0, 0.0};
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < N; k0 += kGemmK) {
    __syncthreads();   // the previous panel is consumed
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      As[idx >> 6][idx & 63] = pa[q];
      Bs[idx & 15][idx >> 4] = pb[q];
    }
    __syncthreads();
    if (k0 + kGemmK < N) fetch(k0 + kGemmK);
#pragma unroll
    for (int ks = 0; ks < kGemmK; ks += 4) {
      double2 av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[ks + lk][wr + 16 * a + li];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[ks + lk][wc + 16 * b + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].x, re[a][b], 0, 0, 0);
          re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[a].y, bv[b].y, re[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].y, im[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[b].x, im[a][b], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = c0 + wc + 16 * b + li;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = r0 + wr + 16 * a + 4 * q + lk;
        if (i < N && j < N) Cb[(int64_t)j * N + i] = double2{re[a][b][q], im[a][b][q]};
      }
    }
}

// Per instance: tau[b] = Tr of column 0 of U (the image of |0><0|, which a
// trace-preserving map keeps at 1); also clears the maxima of the check.
__global__ __launch_bounds__(64) void prop_trace_kernel(const double *U, const int64_t *off4,
                                                        const int32_t *dims, int n_inst,
                                                        double *tau, unsigned long long *dm) {
  const int b = blockIdx.x;
  if (b >= n_inst) return;
  const int n = dims[b];
  const double *c0 = U + 2 * off4[b];
  double sx = 0.0, sy = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) {
    sx += c0[2 * ((int64_t)i * n + i)];
    sy += c0[2 * ((int64_t)i * n + i) + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    sx += __shfl_xor(sx, o);
    sy += __shfl_xor(sy, o);
  }
  if (threadIdx.x == 0) {
    tau[2 * b] = sx;
    tau[2 * b + 1] = sy;
    dm[2 * b] = 0ull;
    dm[2 * b + 1] = 0ull;
  }
}

// U_new /= tau[b] in place, then per instance the largest |U_new - U_old|
// (into dm[2b]) and |U_new| (into dm[2b+1]), as bit patterns of
// non-negative doubles (ordered like the values; NaN above all).
// Grid (blocks, n_inst).
__global__ __launch_bounds__(256) void prop_norm_diff_kernel(double *Un, const double *Uo,
                                                             const int64_t *off4,
                                                             const int32_t *dims,
                                                             const double *tau,
                                                             unsigned long long *dm) {
  const int b = blockIdx.y;
  const int64_t N = (int64_t)dims[b] * dims[b];
  double *x = Un + 2 * off4[b];
  const double *y = Uo + 2 * off4[b];
  const double tr = tau[2 * b], ti = tau[2 * b + 1];
  const double den = tr * tr + ti * ti;
  const double qr = tr / den, qi = -ti / den;   // 1 / tau
  double d = 0.0, m = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N * N;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double ur = x[2 * e], ui = x[2 * e + 1];
    const double vr = ur * qr - ui * qi, vi = ur * qi + ui * qr;
    x[2 * e] = vr;
    x[2 * e + 1] = vi;
    const double dx = vr - y[2 * e], dy = vi - y[2 * e + 1];
    const double v = sqrt(dx * dx + dy * dy), w = sqrt(vr * vr + vi * vi);
    d = (v > d || v != v) ? v : d;   // NaN propagates
    m = (w > m || w != w) ? w : m;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double a = __shfl_xor(d, o), c = __shfl_xor(m, o);
    d = (a > d || a != a) ? a : d;
    m = (c > m || c != c) ? c : m;
  }
  // the four wavefronts' maxima, then one atomic per workgroup and quantity
  __shared__ double wd[4], wm[4];
  if ((threadIdx.x & 63) == 0) {
    wd[threadIdx.x >> 6] = d;
    wm[threadIdx.x >> 6] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      d = (wd[w] > d || wd[w] != wd[w]) ? wd[w] : d;
      m = (wm[w] > m || wm[w] != wm[w]) ? wm[w] : m;
    }
    // |NaN| so that its pattern is the positive quiet NaN, above +inf
    atomicMax(&dm[2 * b], (unsigned long long)__double_as_longlong(d != d ? __builtin_nan("") : d));
    atomicMax(&dm[2 * b + 1],
              (unsigned long long)__double_as_longlong(m != m ? __builtin_nan("") : m));
  }
}

// rho_ss of instance b: column 0 of its limit propagator (the image of
// |0><0|), divided by its trace; packed state layout.
__global__ __launch_bounds__(256) void prop_column0_kernel(const double *U, const int64_t *off4,
                                                           const int32_t *dims,
                                                           const int64_t *off2, double *rho) {
  const int b = blockIdx.x;
  const int n = dims[b];
  const double *c0 = U + 2 * off4[b];      // column 0: the first N entries
  __shared__ double tr[2];
  if (threadIdx.x == 0) {
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < n; ++i) {
      sx += c0[2 * ((int64_t)i * n + i)];
      sy += c0[2 * ((int64_t)i * n + i) + 1];
    }
    tr[0] = sx;
    tr[1] = sy;
  }
  __syncthreads();
  const double den = tr[0] * tr[0] + tr[1] * tr[1];
  double *out = rho + 2 * off2[b];
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    const double x = c0[2 * e], y = c0[2 * e + 1];
    out[2 * e] = (x * tr[0] + y * tr[1]) / den;
    out[2 * e + 1] = (y * tr[0] - x * tr[1]) / den;
  }
}

// status[b] = the first non-zero status of the replicated instances
// [first[b], first[b+1]) (the basis matrices of instance b).
__global__ void range_status_kernel(const int32_t *st, const int64_t *first, int32_t *status,
                                    int n_inst) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_inst) return;
  int v = 0;
  for (int64_t q = first[b]; q < first[b + 1] && v == 0; ++q) v = st[q];
  status[b] = v;
}

}  // namespace

extern "C" hipError_t lme_internal_launch_range_status(const int32_t *st, const int64_t *first,
                                                       int32_t *status, int n_inst,
                                                       hipStream_t s) {
  hipLaunchKernelGGL(range_status_kernel, dim3((n_inst + 255) / 256), dim3(256), 0, s, st, first,
                     status, n_inst);
  return hipGetLastError();
}

extern "C" hipError_t lme_internal_launch_prop_hbasis(double *U, const int64_t *off4,
                                                      const int32_t *dims, int n_inst,
                                                      hipStream_t s) {
  hipLaunchKernelGGL(prop_hbasis_kernel, dim3(256, n_inst), dim3(256), 0, s, U, off4, dims, n_inst);
  return hipGetLastError();
}

extern "C" hipError_t lme_internal_launch_prop_combine(double *U, const int64_t *off4,
                                                       const int32_t *dims, int n_inst,
                                                       hipStream_t s) {
  hipLaunchKernelGGL(prop_combine_kernel, dim3(256, n_inst), dim3(256), 0, s, U, off4, dims,
                     n_inst);
  return hipGetLastError();
}

extern "C" hipError_t lme_internal_launch_zgemm(const void *tiles, int n_tiles, const int64_t *off4,
                                                const int32_t *dims, const double *A,
                                                const double *B, double *C, hipStream_t s) {
  hipLaunchKernelGGL(zgemm_kernel, dim3(n_tiles), dim3(256), 0, s,
                     static_cast<const GemmTile *>(tiles), n_tiles, off4, dims, A, B, C);
  return hipGetLastError();
}

// tau: device double [2 n_inst]; dm: device uint64 [2 n_inst] (the
// maxima as double bit patterns: diff at 2b, magnitude at 2b+1).
extern "C" hipError_t lme_internal_launch_prop_norm_diff(double *Un, const double *Uo,
                                                         const int64_t *off4, const int32_t *dims,
                                                         int n_inst, int64_t max_block,
                                                         double *tau, void *dm, hipStream_t s) {
  unsigned long long *m = static_cast<unsigned long long *>(dm);
  hipLaunchKernelGGL(prop_trace_kernel, dim3(n_inst), dim3(64), 0, s, Un, off4, dims, n_inst, tau,
                     m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // about 16 elements per thread: few enough workgroups that their atomics
  // stay cheap, enough to fill the chip
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>((max_block + 4095) / 4096, 1), 1024);
  hipLaunchKernelGGL(prop_norm_diff_kernel, dim3((unsigned)blocks, n_inst), dim3(256), 0, s, Un,
                     Uo, off4, dims, tau, m);
  return hipGetLastError();
}

extern "C" hipError_t lme_internal_launch_prop_column0(const double *U, const int64_t *off4,
                                                       const int32_t *dims, const int64_t *off2,
                                                       int n_inst, double *rho, hipStream_t s) {
  hipLaunchKernelGGL(prop_column0_kernel, dim3(n_inst), dim3(256), 0, s, U, off4, dims, off2, rho);
  return hipGetLastError();
}
