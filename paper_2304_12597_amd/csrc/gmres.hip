// GPU-resident GMRES (float64) for the capacitance system J_ell x = b
// (Section 2, eq. SMW_linearsystemII).  The paper's own inner solver is a
// FOM-like projection on K_m(K, b) (Section 3, Algorithm 2); by Theorem 1
// J_ell is Hermitian positive definite for SPD K, so any Krylov method
// converges to the same x, and GMRES on J_ell itself needs no extra parfor
// per iteration beyond the product J_ell v_m.
//
// The Arnoldi basis V, the Hessenberg matrix, the Givens rotations and the
// least-squares right-hand side stay in device memory.  Orthogonalisation is
// classical Gram-Schmidt applied twice (CGS2), each pass one multi-block
// kernel with deterministic float64 partial sums.  One small single-block
// kernel per iteration updates the Givens QR and the residual estimate; the
// host reads back 16 bytes per iteration to decide whether to stop.
#include "pd_internal.h"

#include <cmath>

namespace {

constexpr int VB = 256;   // threads per block of the vector kernels

// gm layout (doubles), MX = maxit:
//   H   [MX][MX+1] column-major (H[j*(MX+1) + i])
//   cs  [MX], sn [MX], g [MX+1], y [MX],
//   status [6]: residual estimate, h_{j+1,j}, iterations, beta, converged flag
struct GmLayout {
  int MX;
  __host__ __device__ int H(int i, int j) const { return j * (MX + 1) + i; }
  __host__ __device__ int cs(int j) const { return MX * (MX + 1) + j; }
  __host__ __device__ int sn(int j) const { return MX * (MX + 1) + MX + j; }
  __host__ __device__ int g(int i) const { return MX * (MX + 1) + 2 * MX + i; }
  __host__ __device__ int y(int i) const { return MX * (MX + 1) + 3 * MX + 1 + i; }
  __host__ __device__ int st(int i) const { return MX * (MX + 1) + 4 * MX + 1 + i; }
  __host__ __device__ int size() const { return MX * (MX + 1) + 4 * MX + 1 + 6; }
};
constexpr int GM_DONE = 4;   // status slot of the converged flag

__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) s += sh[w];
  return s;  // valid in thread 0
}

// red[blk*(nv+1) + i] = sum over this block's rows of V_i . w (i < nv) and
// red[blk*(nv+1) + nv] = w . w
__global__ void __launch_bounds__(VB)
dots_kernel(int n, int nv, const double *__restrict__ V, const double *__restrict__ w,
            double *__restrict__ red) {
  __shared__ double sh[VB / 64];
  const int stride = gridDim.x * blockDim.x;
  for (int i = 0; i <= nv; ++i) {
    double s = 0.0;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
      double wr = w[r];
      s += (i < nv ? V[(size_t)i * n + r] : wr) * wr;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) red[blockIdx.x * (nv + 1) + i] = s;
  }
}

// Reduce the partial dots of the previous pass into h (shared), subtract
// V h from w, and (pass < 2) emit the next partial dots.  Block 0 adds h
// into column j of H.
__global__ void __launch_bounds__(VB)
cgs_update_kernel(int n, int nv, int nblk, const double *__restrict__ V, double *__restrict__ w,
                  const double *__restrict__ red_in, double *__restrict__ red_out,
                  double *__restrict__ gm, int MX, int j, int emit) {
  __shared__ double h[128];
  __shared__ double sh[VB / 64];
  GmLayout L{MX};
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += red_in[b * (nv + 1) + i];
    h[i] = s;
  }
  __syncthreads();
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < nv; i += blockDim.x) gm[L.H(i, j)] += h[i];
  const int stride = gridDim.x * blockDim.x;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    double wr = w[r];
    for (int i = 0; i < nv; ++i) wr -= h[i] * V[(size_t)i * n + r];
    w[r] = wr;
  }
  if (!emit) return;
  __syncthreads();
  for (int i = 0; i <= nv; ++i) {
    double s = 0.0;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
      double wr = w[r];
      s += (i < nv ? V[(size_t)i * n + r] : wr) * wr;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) red_out[blockIdx.x * (nv + 1) + i] = s;
  }
}

// Single block: ||w||, Givens update of column j, residual estimate.
// status: [0] = |g_{j+1}| (residual), [1] = h_{j+1,j}, [2] = iterations
__global__ void givens_kernel(int nv, int nblk, const double *__restrict__ red,
                              double *__restrict__ gm, int MX, int j, double *__restrict__ host) {
  GmLayout L{MX};
  if (threadIdx.x != 0) return;
  double nn = 0.0;
  for (int b = 0; b < nblk; ++b) nn += red[b * (nv + 1) + nv];
  double hn = sqrt(nn);
  gm[L.H(j + 1, j)] = hn;
  for (int i = 0; i < j; ++i) {
    double c = gm[L.cs(i)], s = gm[L.sn(i)];
    double a = gm[L.H(i, j)], b = gm[L.H(i + 1, j)];
    gm[L.H(i, j)] = c * a + s * b;
    gm[L.H(i + 1, j)] = -s * a + c * b;
  }
  double a = gm[L.H(j, j)], b = gm[L.H(j + 1, j)];
  double r = hypot(a, b);
  double c = (r == 0.0) ? 1.0 : a / r, s = (r == 0.0) ? 0.0 : b / r;
  gm[L.cs(j)] = c;
  gm[L.sn(j)] = s;
  gm[L.H(j, j)] = r;
  gm[L.H(j + 1, j)] = 0.0;
  double gj = gm[L.g(j)];
  gm[L.g(j)] = c * gj;
  gm[L.g(j + 1)] = -s * gj;
  gm[L.st(0)] = fabs(-s * gj);
  gm[L.st(1)] = hn;
  gm[L.st(2)] = (double)(j + 1);
  host[0] = fabs(-s * gj);
  host[1] = hn;
  host[2] = (double)(j + 1);
  host[3] = gm[L.st(3)];
}

// V_{j+1} = w / ||w|| (or 0 on breakdown); norm taken from status[1]
__global__ void scale_kernel(int n, const double *__restrict__ w, double *__restrict__ out,
                             const double *__restrict__ gm, int MX) {
  GmLayout L{MX};
  double hn = gm[L.st(1)];
  double inv = (hn > 0.0) ? 1.0 / hn : 0.0;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    out[r] = w[r] * inv;
}

// beta = ||b||; g = beta e_1; H = 0; V_0 = b / beta (two launches)
__global__ void init_kernel(int nblk, const double *__restrict__ red, double *__restrict__ gm,
                            int MX, double *__restrict__ host) {
  GmLayout L{MX};
  for (int i = threadIdx.x; i < L.size(); i += blockDim.x) gm[i] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    double nn = 0.0;
    for (int b = 0; b < nblk; ++b) nn += red[b];
    double beta = sqrt(nn);
    gm[L.g(0)] = beta;
    gm[L.st(0)] = beta;
    gm[L.st(1)] = beta;
    gm[L.st(3)] = beta;
    const double done = (beta == 0.0 || !isfinite(beta)) ? 1.0 : 0.0;
    gm[L.st(GM_DONE)] = done;
    host[0] = beta;
    host[1] = beta;
    host[2] = 0.0;
    host[3] = beta;
    host[4] = done;
  }
}

// Back substitution R y = g on the m x m triangle, then x = V y, in one
// launch (m < 0: the iteration count recorded in the status): every block
// reads the (at most 64 x 64) triangle and g into LDS with one parallel round
// trip, solves it on one thread (block 0 also stores y), and forms its rows
// of x.
__global__ void solve_combine_kernel(int n, int m, const double *__restrict__ V,
                                     double *__restrict__ gm, int MX, double *__restrict__ x) {
  __shared__ double Rt[64][65];
  __shared__ double gv[64], yv[64];
  GmLayout L{MX};
  if (m < 0) m = (int)gm[L.st(2)];
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int i = e / m, k = e - i * m;
    if (k >= i) Rt[i][k] = gm[L.H(i, k)];
  }
  for (int i = threadIdx.x; i < m; i += blockDim.x) gv[i] = gm[L.g(i)];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = m - 1; i >= 0; --i) {
      double s = gv[i];
      for (int k = i + 1; k < m; ++k) s -= Rt[i][k] * yv[k];
      const double d = Rt[i][i];
      yv[i] = (d != 0.0) ? s / d : 0.0;
    }
    if (blockIdx.x == 0)
      for (int i = 0; i < m; ++i) gm[L.y(i)] = yv[i];
  }
  __syncthreads();
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += yv[i] * V[(size_t)i * n + r];
    x[r] = s;
  }
}

// ---------------------------------------------------------------------------
// Fused Arnoldi step for vectors of up to 16 * 1024 entries: one block does
// the whole iteration after w = J v_j (two classical Gram-Schmidt passes
// against V_0..V_j, ||w||, the Givens update of column j, the residual
// estimate and V_{j+1} = w / ||w||), with w in registers: row r = tid +
// k*ARN_T of thread tid, RPT rows per thread.  The reduction order depends
// on n only (RPT is fixed by n), so a problem gives the same iterates alone
// and in a batch.  Nothing happens once the converged flag is set; the step
// sets it when the residual estimate reaches rtol * beta, on breakdown
// (h_{j+1,j} = 0) or on a non-finite residual.  st_out[0..3] = residual,
// h_{j+1,j}, iterations, beta; st_out[4] (if with_flag) = converged.
// ---------------------------------------------------------------------------
constexpr int ARN_T = 1024;
constexpr int ARN_MAXN = 16 * ARN_T;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;   // valid in lane 0
}

template <int RPT>
__device__ __forceinline__ void arnoldi_step_body(int n, double *__restrict__ V,
                                                  const double *__restrict__ w,
                                                  double *__restrict__ gm, int MX, int j,
                                                  double rtol, double *__restrict__ st_out,
                                                  bool with_flag) {
  constexpr int NW = ARN_T / 64;
  __shared__ double part[NW][65];
  __shared__ double h[64];
  __shared__ double hcol[66];           // column j of H, accumulated here
  __shared__ double csl[64], snl[64];   // the earlier Givens rotations
  __shared__ double hsh;
  GmLayout L{MX};
  if (gm[L.st(GM_DONE)] != 0.0) return;   // the whole block leaves together
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nv = j + 1;
  // the small state thread 0 needs, read up front in parallel (one global
  // round trip instead of a chain of them); column j of H starts at zero
  if (tid < j) {
    csl[tid] = gm[L.cs(tid)];
    snl[tid] = gm[L.sn(tid)];
  }
  if (tid < j + 2) hcol[tid] = 0.0;
  double gj = 0.0, beta = 0.0;
  if (tid == 0) {
    gj = gm[L.g(j)];
    beta = gm[L.st(3)];
  }
  double wr[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = tid + k * ARN_T;
    wr[k] = r < n ? w[r] : 0.0;
  }
  // the first iterations keep V_0 .. V_j in registers (up to NC vectors,
  // as the register budget allows): each is then read once instead of four
  // times (two passes, each a dot and an update), and a single block's
  // bandwidth is what bounds this step
  constexpr int NC = RPT <= 4 ? 4 : (RPT <= 8 ? 2 : 1);
  const bool cached = RPT <= 8 && nv <= NC;
  double vr[NC][RPT];
  if (cached) {
#pragma unroll
    for (int i = 0; i < NC; ++i)
      if (i < nv) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int r = tid + k * ARN_T;
          vr[i][k] = r < n ? V[(size_t)i * n + r] : 0.0;
        }
      }
  }
  for (int pass = 0; pass < 2; ++pass) {
    if (cached) {
#pragma unroll
      for (int i = 0; i < NC; ++i)
        if (i < nv) {
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < RPT; ++k) {
            const int r = tid + k * ARN_T;
            if (r < n) s += vr[i][k] * wr[k];
          }
          s = wave_sum(s);
          if (lane == 0) part[wv][i] = s;
        }
    } else {
      for (int i = 0; i < nv; ++i) {
        const double *vi = V + (size_t)i * n;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int r = tid + k * ARN_T;
          if (r < n) s += vi[r] * wr[k];
        }
        s = wave_sum(s);
        if (lane == 0) part[wv][i] = s;
      }
    }
    __syncthreads();
    if (tid < nv) {
      double s = 0.0;
      for (int q = 0; q < NW; ++q) s += part[q][tid];
      h[tid] = s;
      hcol[tid] += s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = tid + k * ARN_T;
      if (r < n) {
        double t = wr[k];
        if (cached) {
#pragma unroll
          for (int i = 0; i < NC; ++i)
            if (i < nv) t -= h[i] * vr[i][k];
        } else {
          for (int i = 0; i < nv; ++i) t -= h[i] * V[(size_t)i * n + r];
        }
        wr[k] = t;
      }
    }
    __syncthreads();   // part is written again
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) s += wr[k] * wr[k];
  s = wave_sum(s);
  if (lane == 0) part[wv][0] = s;
  __syncthreads();
  if (tid == 0) {
    double nn = 0.0;
    for (int q = 0; q < NW; ++q) nn += part[q][0];
    const double hn = sqrt(nn);
    hcol[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double c = csl[i], sn = snl[i];
      const double a = hcol[i], b = hcol[i + 1];
      hcol[i] = c * a + sn * b;
      hcol[i + 1] = -sn * a + c * b;
    }
    const double a = hcol[j], b = hcol[j + 1];
    const double rr = hypot(a, b);
    const double c = (rr == 0.0) ? 1.0 : a / rr, sn = (rr == 0.0) ? 0.0 : b / rr;
    gm[L.cs(j)] = c;
    gm[L.sn(j)] = sn;
    hcol[j] = rr;
    hcol[j + 1] = 0.0;
    gm[L.g(j)] = c * gj;
    gm[L.g(j + 1)] = -sn * gj;
    const double res = fabs(-sn * gj);
    const double done = (res <= rtol * beta || hn == 0.0 || !isfinite(res)) ? 1.0 : 0.0;
    gm[L.st(0)] = res;
    gm[L.st(1)] = hn;
    gm[L.st(2)] = (double)(j + 1);
    gm[L.st(GM_DONE)] = done;
    st_out[0] = res;
    st_out[1] = hn;
    st_out[2] = (double)(j + 1);
    st_out[3] = beta;
    if (with_flag) st_out[4] = done;
    hsh = hn;
  }
  __syncthreads();
  if (tid < j + 2) gm[L.H(tid, j)] = hcol[tid];
  const double inv = (hsh > 0.0) ? 1.0 / hsh : 0.0;
  double *vn = V + (size_t)(j + 1) * n;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = tid + k * ARN_T;
    if (r < n) vn[r] = wr[k] * inv;
  }
}

template <int RPT>
__global__ void __launch_bounds__(ARN_T)
arnoldi_step_kernel(int n, double *__restrict__ V, const double *__restrict__ w,
                    double *__restrict__ gm, int MX, int j, double rtol,
                    double *__restrict__ host) {
  arnoldi_step_body<RPT>(n, V, w, gm, MX, j, rtol, host, true);
}

}  // namespace

size_t pd_gmres_state_doubles(int maxit) { return (size_t)GmLayout{maxit}.size(); }

int pd_vec_blocks(int n) {
  int b = (n + VB - 1) / VB;
  return b < 256 ? b : 256;
}

namespace {

// Start of GMRES on one block: beta = ||b||, the small state reset (g =
// beta e_1, converged flag set when beta is 0 or not finite), V_0 = b / beta.
// st_out[0..3] = beta, beta, 0, beta; st_out[4] (with_flag) = converged.
template <int RPT>
__device__ __forceinline__ void gm_init_body(int n, const double *__restrict__ b,
                                             double *__restrict__ V, double *__restrict__ gm,
                                             int MX, double *__restrict__ st_out, bool with_flag) {
  constexpr int NW = ARN_T / 64;
  __shared__ double part[NW];
  __shared__ double bsh;
  GmLayout L{MX};
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < L.size(); i += blockDim.x) gm[i] = 0.0;
  double br[RPT];
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = tid + k * ARN_T;
    br[k] = r < n ? b[r] : 0.0;
    s += br[k] * br[k];
  }
  s = wave_sum(s);
  if (lane == 0) part[wv] = s;
  __syncthreads();   // also orders the reset of gm before thread 0 writes it
  if (tid == 0) {
    double nn = 0.0;
    for (int q = 0; q < NW; ++q) nn += part[q];
    const double beta = sqrt(nn);
    const double done = (beta == 0.0 || !isfinite(beta)) ? 1.0 : 0.0;
    gm[L.g(0)] = beta;
    gm[L.st(0)] = beta;
    gm[L.st(1)] = beta;
    gm[L.st(3)] = beta;
    gm[L.st(GM_DONE)] = done;
    st_out[0] = beta;
    st_out[1] = beta;
    st_out[2] = 0.0;
    st_out[3] = beta;
    if (with_flag) st_out[4] = done;
    bsh = beta;
  }
  __syncthreads();
  const double inv = (bsh > 0.0) ? 1.0 / bsh : 0.0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = tid + k * ARN_T;
    if (r < n) V[r] = br[k] * inv;
  }
}

template <int RPT>
__global__ void __launch_bounds__(ARN_T)
gm_init_kernel(int n, const double *__restrict__ b, double *__restrict__ V,
               double *__restrict__ gm, int MX, double *__restrict__ host) {
  gm_init_body<RPT>(n, b, V, gm, MX, host, true);
}

void launch_gm_init(pd_plan p, const double *b) {
  const int n = p->ncap;
  if (n <= 4 * ARN_T)
    hipLaunchKernelGGL((gm_init_kernel<4>), dim3(1), dim3(ARN_T), 0, p->stream, n, b, p->V,
                       p->gm, p->maxit, p->host_dev);
  else if (n <= 8 * ARN_T)
    hipLaunchKernelGGL((gm_init_kernel<8>), dim3(1), dim3(ARN_T), 0, p->stream, n, b, p->V,
                       p->gm, p->maxit, p->host_dev);
  else
    hipLaunchKernelGGL((gm_init_kernel<16>), dim3(1), dim3(ARN_T), 0, p->stream, n, b, p->V,
                       p->gm, p->maxit, p->host_dev);
}

void launch_arnoldi(pd_plan p, int j, double rtol) {
  const int n = p->ncap;
  GmLayout L{p->maxit};
  (void)L;
  if (n <= 4 * ARN_T)
    hipLaunchKernelGGL((arnoldi_step_kernel<4>), dim3(1), dim3(ARN_T), 0, p->stream, n, p->V,
                       p->wvec, p->gm, p->maxit, j, rtol, p->host_dev);
  else if (n <= 8 * ARN_T)
    hipLaunchKernelGGL((arnoldi_step_kernel<8>), dim3(1), dim3(ARN_T), 0, p->stream, n, p->V,
                       p->wvec, p->gm, p->maxit, j, rtol, p->host_dev);
  else
    hipLaunchKernelGGL((arnoldi_step_kernel<16>), dim3(1), dim3(ARN_T), 0, p->stream, n, p->V,
                       p->wvec, p->gm, p->maxit, j, rtol, p->host_dev);
}

// Enqueues (no synchronisation) J v_j and the fused Arnoldi step for
// iterations j0 .. j0 + count - 1, the capacitance kernels reading the
// converged flag.
pd_status enqueue_iters(pd_plan p, int j0, int count, double rtol) {
  GmLayout L{p->maxit};
  const int n = p->ncap;
  p->gm_skip = p->gm + L.st(GM_DONE);
  pd_status s = PD_OK;
  for (int j = j0; j < j0 + count && j < p->maxit && s == PD_OK; ++j) {
    s = pd_capacitance_apply_impl(p, p->V + (size_t)j * n, p->wvec);
    if (s == PD_OK) launch_arnoldi(p, j, rtol);
  }
  p->gm_skip = nullptr;
  if (s != PD_OK) return s;
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

// 1D plans: fused Arnoldi steps enqueued in chunks (2, 4, then 8 iterations)
// with one stream synchronisation per chunk; once the device-side converged
// flag is set, the remaining launches of a chunk return at once (the
// capacitance product's kernels read the flag through p->gm_skip).
pd_status gmres_fused(pd_plan p, const double *b, double *x, double rtol, int *iters,
                      double *relres) {
  const int n = p->ncap, MX = p->maxit;
  const int B = pd_vec_blocks(n);
  GmLayout L{MX};
  volatile double *st = p->host_pin;
  launch_gm_init(p, b);
  PD_HIP_CHECK(hipGetLastError());
  p->gm_skip = p->gm + L.st(GM_DONE);
  int j = 0, chunk = 2;
  pd_status s = PD_OK;
  bool done = false;
  while (j < MX && !done) {
    const int c = (chunk < MX - j) ? chunk : MX - j;
    for (int t = 0; t < c && s == PD_OK; ++t, ++j) {
      s = pd_capacitance_apply_impl(p, p->V + (size_t)j * n, p->wvec);
      if (s == PD_OK) {
        launch_arnoldi(p, j, rtol);
        if (hipGetLastError() != hipSuccess) s = PD_EHIP;
      }
    }
    if (s != PD_OK) break;
    if (hipStreamSynchronize(p->stream) != hipSuccess) {
      s = PD_EHIP;
      break;
    }
    done = st[4] != 0.0;
    chunk = chunk < 8 ? 2 * chunk : 8;
  }
  p->gm_skip = nullptr;
  if (s == PD_EHIP) {
    pd_set_error("capacitance GMRES: HIP error");
    return s;
  }
  if (s != PD_OK) return s;
  const double beta = st[3];
  if (!std::isfinite(beta)) {
    pd_set_error("capacitance right-hand side is not finite");
    return PD_ENONFINITE;
  }
  const int m = (int)st[2];
  const double res = st[0];
  if (!std::isfinite(res)) {
    pd_set_error("capacitance GMRES produced a non-finite residual");
    return PD_ENONFINITE;
  }
  if (beta == 0.0) {
    PD_HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * n, p->stream));
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return PD_OK;
  }
  hipLaunchKernelGGL(solve_combine_kernel, dim3(B), dim3(VB), 0, p->stream, n, m, p->V, p->gm, MX,
                     x);
  PD_HIP_CHECK(hipGetLastError());
  if (iters) *iters = m;
  if (relres) *relres = res / beta;
  return (res <= rtol * beta || st[1] == 0.0) ? PD_OK : PD_ENOTCONV;
}

}  // namespace

bool pd_gmres_fused_ok(pd_plan p) { return p->dims == 1 && p->ncap <= ARN_MAXN; }
size_t pd_gmres_done_index(int maxit) { return (size_t)GmLayout{maxit}.st(GM_DONE); }

// Speculative form: init, `count` iterations and x = V y with the iteration
// count taken from the device status, all enqueued without synchronising.
pd_status pd_gmres_enqueue(pd_plan p, const double *b, double *x, double rtol, int count) {
  const int n = p->ncap, MX = p->maxit;
  const int B = pd_vec_blocks(n);
  launch_gm_init(p, b);
  PD_HIP_CHECK(hipGetLastError());
  pd_status s = enqueue_iters(p, 0, count, rtol);
  if (s != PD_OK) return s;
  hipLaunchKernelGGL(solve_combine_kernel, dim3(B), dim3(VB), 0, p->stream, n, -1, p->V, p->gm, MX,
                     x);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

// After a synchronisation: the status of the speculative GMRES.
void pd_gmres_read(pd_plan p, int *m, double *res, double *beta, bool *done) {
  volatile double *st = p->host_pin;
  *res = st[0];
  *beta = st[3];
  *m = (int)st[2];
  *done = st[4] != 0.0;
}

// Continues a speculative GMRES that had not converged (iterations from m on,
// one synchronisation per chunk), then x = V y.  Returns the final status.
pd_status pd_gmres_continue(pd_plan p, double *x, double rtol, int *iters, double *relres) {
  const int n = p->ncap, MX = p->maxit;
  const int B = pd_vec_blocks(n);
  volatile double *st = p->host_pin;
  int j = (int)st[2], chunk = 2;
  bool done = st[4] != 0.0;
  while (j < MX && !done) {
    const int c = (chunk < MX - j) ? chunk : MX - j;
    pd_status s = enqueue_iters(p, j, c, rtol);
    if (s != PD_OK) return s;
    j += c;
    PD_HIP_CHECK(hipStreamSynchronize(p->stream));
    done = st[4] != 0.0;
    chunk = chunk < 8 ? 2 * chunk : 8;
  }
  const int m = (int)st[2];
  const double res = st[0], beta = st[3];
  if (!std::isfinite(res)) {
    pd_set_error("capacitance GMRES produced a non-finite residual");
    return PD_ENONFINITE;
  }
  hipLaunchKernelGGL(solve_combine_kernel, dim3(B), dim3(VB), 0, p->stream, n, m, p->V, p->gm, MX,
                     x);
  PD_HIP_CHECK(hipGetLastError());
  if (iters) *iters = m;
  if (relres) *relres = beta > 0.0 ? res / beta : 0.0;
  return (res <= rtol * beta || st[1] == 0.0) ? PD_OK : PD_ENOTCONV;
}

pd_status pd_gmres(pd_plan p, const double *b, double *x, double rtol, int *iters,
                   double *relres) {
  if (p->dims == 1 && p->ncap <= ARN_MAXN) return gmres_fused(p, b, x, rtol, iters, relres);
  const int n = p->ncap, MX = p->maxit;
  const int B = pd_vec_blocks(n);
  GmLayout L{MX};
  double *red1 = p->red, *red2 = p->red + (size_t)B * (MX + 2);
  double *st_host = p->host_pin;
  // beta = ||b||
  hipLaunchKernelGGL(dots_kernel, dim3(B), dim3(VB), 0, p->stream, n, 0, p->V, b, red1);
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(256), 0, p->stream, B, red1, p->gm, MX,
                     p->host_dev);
  hipLaunchKernelGGL(scale_kernel, dim3(B), dim3(VB), 0, p->stream, n, b, p->V, p->gm, MX);
  PD_HIP_CHECK(hipGetLastError());
  PD_HIP_CHECK(hipStreamSynchronize(p->stream));
  const double beta = ((volatile double *)st_host)[0];
  if (!std::isfinite(beta)) {
    pd_set_error("capacitance right-hand side is not finite");
    return PD_ENONFINITE;
  }
  if (beta == 0.0) {
    PD_HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * n, p->stream));
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return PD_OK;
  }
  int m = 0;
  double res = beta;
  for (int j = 0; j < MX; ++j) {
    const double *vj = p->V + (size_t)j * n;
    pd_status s = pd_capacitance_apply_impl(p, vj, p->wvec);
    if (s != PD_OK) return s;
    // CGS2: dots, update+dots, update
    hipLaunchKernelGGL(dots_kernel, dim3(B), dim3(VB), 0, p->stream, n, j + 1, p->V, p->wvec,
                       red1);
    hipLaunchKernelGGL(cgs_update_kernel, dim3(B), dim3(VB), 0, p->stream, n, j + 1, B, p->V,
                       p->wvec, red1, red2, p->gm, MX, j, 1);
    hipLaunchKernelGGL(cgs_update_kernel, dim3(B), dim3(VB), 0, p->stream, n, j + 1, B, p->V,
                       p->wvec, red2, red1, p->gm, MX, j, 0);
    hipLaunchKernelGGL(dots_kernel, dim3(B), dim3(VB), 0, p->stream, n, 0, p->V, p->wvec, red1);
    hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(64), 0, p->stream, 0, B, red1, p->gm, MX,
                       j, p->host_dev);
    hipLaunchKernelGGL(scale_kernel, dim3(B), dim3(VB), 0, p->stream, n, p->wvec,
                       p->V + (size_t)(j + 1) * n, p->gm, MX);
    PD_HIP_CHECK(hipGetLastError());
    PD_HIP_CHECK(hipStreamSynchronize(p->stream));
    m = j + 1;
    res = ((volatile double *)st_host)[0];
    if (!std::isfinite(res)) {
      pd_set_error("capacitance GMRES produced a non-finite residual");
      return PD_ENONFINITE;
    }
    if (res <= rtol * beta || ((volatile double *)st_host)[1] == 0.0) break;
  }
  hipLaunchKernelGGL(solve_combine_kernel, dim3(B), dim3(VB), 0, p->stream, n, m, p->V, p->gm, MX,
                     x);
  PD_HIP_CHECK(hipGetLastError());
  if (iters) *iters = m;
  if (relres) *relres = res / beta;
  return (res <= rtol * beta || ((volatile double *)st_host)[1] == 0.0) ? PD_OK : PD_ENOTCONV;
}

// ---------------------------------------------------------------------------
// Batched GMRES: the same steps for many independent problems in lockstep
// (iteration j is shared); problems whose flag in `active` is 0 are skipped.
// ---------------------------------------------------------------------------
namespace {

// which = 0: dots of w with V_0..V_{nv-1} and w.w into red1;
// which = 1: ||b||^2 into red1 (nv = 0)
__global__ void __launch_bounds__(VB)
batch_dots_kernel(const VecJob *__restrict__ jobs, const int2 *__restrict__ vmap, int nv,
                  int which, const int *__restrict__ active) {
  __shared__ double sh[VB / 64];
  const int2 m = vmap[blockIdx.x];
  if (active && !active[m.x]) return;
  const VecJob &J = jobs[m.x];
  const double *w = which ? J.b : J.w;
  const int n = J.n;
  const int stride = J.B * blockDim.x;
  for (int i = 0; i <= nv; ++i) {
    double s = 0.0;
    for (int r = m.y * blockDim.x + threadIdx.x; r < n; r += stride) {
      const double wr = w[r];
      s += (i < nv ? J.V[(size_t)i * n + r] : wr) * wr;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) J.red1[m.y * (nv + 1) + i] = s;
  }
}

// pass 1: h from red1, w -= V h, dots into red2;  pass 2: h from red2, w -= V h
__global__ void __launch_bounds__(VB)
batch_update_kernel(const VecJob *__restrict__ jobs, const int2 *__restrict__ vmap, int nv, int j,
                    int MX, int pass, const int *__restrict__ active) {
  __shared__ double h[128];
  __shared__ double sh[VB / 64];
  const int2 m = vmap[blockIdx.x];
  if (active && !active[m.x]) return;
  const VecJob &J = jobs[m.x];
  GmLayout L{MX};
  const double *red_in = (pass == 1) ? J.red1 : J.red2;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < J.B; ++b) s += red_in[b * (nv + 1) + i];
    h[i] = s;
  }
  __syncthreads();
  if (m.y == 0)
    for (int i = threadIdx.x; i < nv; i += blockDim.x) J.gm[L.H(i, j)] += h[i];
  const int n = J.n;
  const int stride = J.B * blockDim.x;
  for (int r = m.y * blockDim.x + threadIdx.x; r < n; r += stride) {
    double wr = J.w[r];
    for (int i = 0; i < nv; ++i) wr -= h[i] * J.V[(size_t)i * n + r];
    J.w[r] = wr;
  }
  if (pass != 1) return;
  __syncthreads();
  for (int i = 0; i <= nv; ++i) {
    double s = 0.0;
    for (int r = m.y * blockDim.x + threadIdx.x; r < n; r += stride) {
      const double wr = J.w[r];
      s += (i < nv ? J.V[(size_t)i * n + r] : wr) * wr;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) J.red2[m.y * (nv + 1) + i] = s;
  }
}

// one block per problem: ||w|| from red1 (nv = 0 layout), Givens update;
// status[4*p + 0..3] = residual, h_{j+1,j}, iterations, beta
__global__ void batch_givens_kernel(const VecJob *__restrict__ jobs, int j, int MX,
                                    double *__restrict__ status, const int *__restrict__ active) {
  const int p = blockIdx.x;
  if (threadIdx.x != 0 || (active && !active[p])) return;
  const VecJob &J = jobs[p];
  double *gm = J.gm;
  GmLayout L{MX};
  double nn = 0.0;
  for (int b = 0; b < J.B; ++b) nn += J.red1[b];
  const double hn = sqrt(nn);
  gm[L.H(j + 1, j)] = hn;
  for (int i = 0; i < j; ++i) {
    const double c = gm[L.cs(i)], s = gm[L.sn(i)];
    const double a = gm[L.H(i, j)], b = gm[L.H(i + 1, j)];
    gm[L.H(i, j)] = c * a + s * b;
    gm[L.H(i + 1, j)] = -s * a + c * b;
  }
  const double a = gm[L.H(j, j)], b = gm[L.H(j + 1, j)];
  const double r = hypot(a, b);
  const double c = (r == 0.0) ? 1.0 : a / r, s = (r == 0.0) ? 0.0 : b / r;
  gm[L.cs(j)] = c;
  gm[L.sn(j)] = s;
  gm[L.H(j, j)] = r;
  gm[L.H(j + 1, j)] = 0.0;
  const double gj = gm[L.g(j)];
  gm[L.g(j)] = c * gj;
  gm[L.g(j + 1)] = -s * gj;
  gm[L.st(0)] = fabs(-s * gj);
  gm[L.st(1)] = hn;
  gm[L.st(2)] = (double)(j + 1);
  status[4 * p + 0] = fabs(-s * gj);
  status[4 * p + 1] = hn;
  status[4 * p + 2] = (double)(j + 1);
  status[4 * p + 3] = gm[L.st(3)];
}

// one block per problem: reset the small state, beta = ||b|| from red1
__global__ void batch_init_kernel(const VecJob *__restrict__ jobs, int MX,
                                  double *__restrict__ status) {
  const VecJob &J = jobs[blockIdx.x];
  GmLayout L{MX};
  for (int i = threadIdx.x; i < L.size(); i += blockDim.x) J.gm[i] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    double nn = 0.0;
    for (int b = 0; b < J.B; ++b) nn += J.red1[b];
    const double beta = sqrt(nn);
    J.gm[L.g(0)] = beta;
    J.gm[L.st(0)] = beta;
    J.gm[L.st(1)] = beta;
    J.gm[L.st(3)] = beta;
    J.gm[L.st(GM_DONE)] = (beta == 0.0 || !isfinite(beta)) ? 1.0 : 0.0;
    status[4 * blockIdx.x + 0] = beta;
    status[4 * blockIdx.x + 1] = beta;
    status[4 * blockIdx.x + 2] = 0.0;
    status[4 * blockIdx.x + 3] = beta;
  }
}

// V_{j+1} = w / h_{j+1,j} (from_b: V_0 = b / beta)
__global__ void batch_scale_kernel(const VecJob *__restrict__ jobs, const int2 *__restrict__ vmap,
                                   int j, int MX, int from_b, const int *__restrict__ active) {
  const int2 m = vmap[blockIdx.x];
  if (active && !active[m.x]) return;
  const VecJob &J = jobs[m.x];
  GmLayout L{MX};
  const double hn = J.gm[L.st(1)];
  const double inv = (hn > 0.0) ? 1.0 / hn : 0.0;
  const double *src = from_b ? J.b : J.w;
  double *dst = J.V + (size_t)(from_b ? 0 : j + 1) * J.n;
  for (int r = m.y * blockDim.x + threadIdx.x; r < J.n; r += J.B * blockDim.x)
    dst[r] = src[r] * inv;
}

// one block per problem: the fused Arnoldi step (same body as the single
// problem's, rows per thread fixed by the problem's n)
__global__ void __launch_bounds__(ARN_T)
batch_arnoldi_kernel(const VecJob *__restrict__ jobs, int j, int MX, double rtol,
                     double *__restrict__ status, const int *__restrict__ active) {
  const int p = blockIdx.x;
  if (active && !active[p]) return;
  const VecJob &J = jobs[p];
  double *st = status + 4 * p;
  if (J.n <= 4 * ARN_T)
    arnoldi_step_body<4>(J.n, J.V, J.w, J.gm, MX, j, rtol, st, false);
  else if (J.n <= 8 * ARN_T)
    arnoldi_step_body<8>(J.n, J.V, J.w, J.gm, MX, j, rtol, st, false);
  else
    arnoldi_step_body<16>(J.n, J.V, J.w, J.gm, MX, j, rtol, st, false);
}

// one block per problem: the fused start of GMRES (same body as alone)
__global__ void __launch_bounds__(ARN_T)
batch_gm_init_kernel(const VecJob *__restrict__ jobs, int MX, double *__restrict__ status) {
  const VecJob &J = jobs[blockIdx.x];
  double *st = status + 4 * blockIdx.x;
  if (J.n <= 4 * ARN_T)
    gm_init_body<4>(J.n, J.b, J.V, J.gm, MX, st, false);
  else if (J.n <= 8 * ARN_T)
    gm_init_body<8>(J.n, J.b, J.V, J.gm, MX, st, false);
  else
    gm_init_body<16>(J.n, J.b, J.V, J.gm, MX, st, false);
}

// per problem: back substitution (block 0 of the problem does it first in a
// separate launch), then x = V y
__global__ void batch_backsolve_kernel(const VecJob *__restrict__ jobs, int MX,
                                       const int *__restrict__ mlist) {
  const VecJob &J = jobs[blockIdx.x];
  if (threadIdx.x != 0) return;
  GmLayout L{MX};
  const int m = mlist ? mlist[blockIdx.x] : (int)J.gm[L.st(2)];
  double *gm = J.gm;
  for (int i = m - 1; i >= 0; --i) {
    double s = gm[L.g(i)];
    for (int k = i + 1; k < m; ++k) s -= gm[L.H(i, k)] * gm[L.y(k)];
    const double d = gm[L.H(i, i)];
    gm[L.y(i)] = (d != 0.0) ? s / d : 0.0;
  }
}

__global__ void batch_combine_kernel(const VecJob *__restrict__ jobs, const int2 *__restrict__ vmap,
                                     int MX, const int *__restrict__ mlist) {
  const int2 mp = vmap[blockIdx.x];
  const VecJob &J = jobs[mp.x];
  GmLayout L{MX};
  const int m = mlist ? mlist[mp.x] : (int)J.gm[L.st(2)];
  for (int r = mp.y * blockDim.x + threadIdx.x; r < J.n; r += J.B * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += J.gm[L.y(i)] * J.V[(size_t)i * J.n + r];
    J.x[r] = s;
  }
}

}  // namespace

pd_status pd_gmres_batch_dots(const VecJob *jobs, const int2 *vmap, int nvb, int nv, int which,
                              const int *active, hipStream_t s) {
  hipLaunchKernelGGL(batch_dots_kernel, dim3(nvb), dim3(VB), 0, s, jobs, vmap, nv, which, active);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

pd_status pd_gmres_batch_update(const VecJob *jobs, const int2 *vmap, int nvb, int nv, int j,
                                int MX, int pass, const int *active, hipStream_t s) {
  hipLaunchKernelGGL(batch_update_kernel, dim3(nvb), dim3(VB), 0, s, jobs, vmap, nv, j, MX, pass,
                     active);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

pd_status pd_gmres_batch_arnoldi(const VecJob *jobs, int count, int j, int MX, double rtol,
                                 double *status, const int *active, hipStream_t s) {
  hipLaunchKernelGGL(batch_arnoldi_kernel, dim3(count), dim3(ARN_T), 0, s, jobs, j, MX, rtol,
                     status, active);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

int pd_gmres_fused_max_n() { return ARN_MAXN; }

pd_status pd_gmres_batch_start(const VecJob *jobs, int count, int MX, double *status,
                               hipStream_t s) {
  hipLaunchKernelGGL(batch_gm_init_kernel, dim3(count), dim3(ARN_T), 0, s, jobs, MX, status);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

pd_status pd_gmres_batch_givens(const VecJob *jobs, int count, int j, int MX, double *status,
                                const int *active, hipStream_t s) {
  hipLaunchKernelGGL(batch_givens_kernel, dim3(count), dim3(64), 0, s, jobs, j, MX, status,
                     active);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

pd_status pd_gmres_batch_init(const VecJob *jobs, int count, int MX, double *status,
                              hipStream_t s) {
  hipLaunchKernelGGL(batch_init_kernel, dim3(count), dim3(256), 0, s, jobs, MX, status);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

pd_status pd_gmres_batch_scale(const VecJob *jobs, const int2 *vmap, int nvb, int j, int MX,
                               int from_b, const int *active, hipStream_t s) {
  hipLaunchKernelGGL(batch_scale_kernel, dim3(nvb), dim3(VB), 0, s, jobs, vmap, j, MX, from_b,
                     active);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

pd_status pd_gmres_batch_finish(const VecJob *jobs, const int2 *vmap, int nvb, int count, int MX,
                                const int *m_per_problem, hipStream_t s) {
  hipLaunchKernelGGL(batch_backsolve_kernel, dim3(count), dim3(64), 0, s, jobs, MX, m_per_problem);
  hipLaunchKernelGGL(batch_combine_kernel, dim3(nvb), dim3(VB), 0, s, jobs, vmap, MX,
                     m_per_problem);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}
