// lme_corr.hip -- the step between the two evolutions of a two-time
// correlation function (quantum regression theorem): sigma_{b,i} = B_b rho_b(t_i)
// for every instance b and first time t_i, written in the packed layout of
// the replicated batch that the second evolution integrates.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

struct __attribute__((aligned(16))) cplx {
  double x, y;
};

__device__ inline cplx cfma(cplx a, cplx b, cplx c) {
  return {fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}

struct LeftMulArgs {
  int32_t n_inst, n_t, wB;
  int64_t state_elems;        // elements of one state copy of the batch
  const int64_t *off;         // [n_inst] packed offsets of the batch
  const int32_t *dims;        // [n_inst]
  const int64_t *boff;        // [n_inst] offsets into the B pool (entries)
  const cplx *Bval;           // pool: per instance [wB][n] values
  const int32_t *Bcol;        // pool: per instance [wB][n] columns (padding: value 0)
  const cplx *states;         // [n_t][state_elems]: rho(t_i)
  cplx *sigma;                // replicated batch: instance b*n_t + i at n_t*off[b] + i*n^2
};

// One workgroup per (instance, first time): sigma = B rho(t_i), every
// element (row, col) from the wB entries of row `row` of B.
__global__ __launch_bounds__(256) void left_mul_kernel(LeftMulArgs a) {
  const int r = blockIdx.x;
  const int b = r / a.n_t, i = r - b * a.n_t;
  const int n = a.dims[b];
  const int64_t n2 = (int64_t)n * n;
  const cplx *rho = a.states + (int64_t)i * a.state_elems + a.off[b];
  cplx *sig = a.sigma + (int64_t)a.n_t * a.off[b] + (int64_t)i * n2;
  const cplx *bv = a.Bval + a.boff[b];
  const int32_t *bc = a.Bcol + a.boff[b];
  for (int64_t e = threadIdx.x; e < n2; e += blockDim.x) {
    const int row = (int)(e / n), col = (int)(e - (int64_t)row * n);
    cplx acc = {0.0, 0.0};
    for (int s = 0; s < a.wB; ++s)
      acc = cfma(bv[s * n + row], rho[(int64_t)bc[s * n + row] * n + col], acc);
    sig[e] = acc;
  }
}

// status[b] = the first failure of instance b: its first evolution, then its
// second evolutions in order of the first time.
__global__ void corr_status_kernel(const int32_t *st1, const int32_t *st2, int32_t *status,
                                   int n_inst, int n_t) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_inst) return;
  int s = st1[b];
  for (int i = 0; i < n_t && s == 0; ++i) s = st2[(int64_t)b * n_t + i];
  status[b] = s;
}

}  // namespace

extern "C" hipError_t lme_internal_launch_left_mul(int n_inst, int n_t, int wB, int64_t state_elems,
                                                   const int64_t *off, const int32_t *dims,
                                                   const int64_t *boff, const double *Bval,
                                                   const int32_t *Bcol, const double *states,
                                                   double *sigma, hipStream_t s) {
  LeftMulArgs a;
  a.n_inst = n_inst;
  a.n_t = n_t;
  a.wB = wB;
  a.state_elems = state_elems;
  a.off = off;
  a.dims = dims;
  a.boff = boff;
  a.Bval = reinterpret_cast<const cplx *>(Bval);
  a.Bcol = Bcol;
  a.states = reinterpret_cast<const cplx *>(states);
  a.sigma = reinterpret_cast<cplx *>(sigma);
  hipLaunchKernelGGL(left_mul_kernel, dim3((unsigned)(n_inst * n_t)), dim3(256), 0, s, a);
  return hipGetLastError();
}

extern "C" hipError_t lme_internal_launch_corr_status(const int32_t *st1, const int32_t *st2,
                                                      int32_t *status, int n_inst, int n_t,
                                                      hipStream_t s) {
  hipLaunchKernelGGL(corr_status_kernel, dim3((n_inst + 255) / 256), dim3(256), 0, s, st1, st2,
                     status, n_inst, n_t);
  return hipGetLastError();
}
