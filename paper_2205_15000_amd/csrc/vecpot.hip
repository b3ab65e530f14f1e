// Induced vector potential with the separable, eigen-truncated kernel of
// App. D, and the magnetic moment of Sec. V.A (Eq. magnetic_moment_def).
//
// With G = V Lambda V^T kept to N* modes, A = -kappa^-2 sum_k lambda_k
// T_k J' T_k, where T_k[a][b] = V_k[|a - b|] is a symmetric Toeplitz
// matrix.  Two FP64 MFMA contractions per component:
//   Y_k = J' T_k        (one N x N x N product per mode; T_k generated from V_k),
//   A   = s sum_k lambda_k T_k Y_k   (one N x (N* N) x N product; lambda_k T_k
//                        generated from V_k, Y stacked mode by mode).
// The Toeplitz operands are formed from the N-vector of each mode as they
// are staged into LDS, so no N x N x N* table is stored.
#include "kernels.hpp"
#include "sweep.hpp"

namespace qc {

typedef double v4d __attribute__((ext_vector_type(4)));

// One wave per 32 x 32 output tile (2 x 2 MFMA 16x16x4 tiles), K staged
// through LDS in chunks of 16.  MFMA f64 16x16x4 operands: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; the result D[l / 16 + 4 v][l % 16]
// in element v of its four accumulators (checked on the device).
//   MODE 1: C = Y[c][k] (N x N), A = J'[c] (row-major), B[a][b] = V[k][|a - b|];
//           blockIdx.z = c * nmodes + k.
//   MODE 2: C = A_out[c], A[r][(k, a)] = lambda_k V[k][|r - a|],
//           B = Y[c] as an (N* N) x N row-major matrix; blockIdx.z = c.
template <int MODE>
__global__ void __launch_bounds__(64) eig_gemm_kernel(int n, int nmodes, const double* __restrict__ jp,
                                                      const double* __restrict__ vk,
                                                      const double* __restrict__ lam, double* __restrict__ y,
                                                      double* __restrict__ aout, double alpha) {
  __shared__ double As[16][33];  // [k][row]
  __shared__ double Bs[16][33];  // [k][col]
  const int l = threadIdx.x;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int z = blockIdx.z;
  const int64_t nn = static_cast<int64_t>(n) * n;
  const int K = MODE == 1 ? n : nmodes * n;
  const double* aptr = nullptr;
  const double* bptr = nullptr;
  const double* vrow = nullptr;
  double* cptr = nullptr;
  if (MODE == 1) {
    const int c = z / nmodes, k = z - (z / nmodes) * nmodes;
    aptr = jp + c * nn;
    vrow = vk + static_cast<int64_t>(k) * n;
    cptr = y + static_cast<int64_t>(z) * nn;
  } else {
    bptr = y + static_cast<int64_t>(z) * nmodes * nn;
    cptr = aout + static_cast<int64_t>(z) * nn;
  }
  v4d acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int kb = 0; kb < K; kb += 16) {
    // stage A (32 rows x 16 k) and B (16 k x 32 cols): 8 elements per lane each
    for (int e = 0; e < 8; ++e) {
      const int idx = e * 64 + l;
      {  // A: row ar, k ak (k fastest across lanes)
        const int ar = idx >> 4, ak = idx & 15;
        const int r = r0 + ar, q = kb + ak;
        double v = 0.0;
        if (r < n && q < K) {
          if (MODE == 1) {
            v = aptr[static_cast<int64_t>(r) * n + q];
          } else {
            const int k = q / n, a = q - k * n;
            const int d = r > a ? r - a : a - r;
            v = lam[k] * vk[static_cast<int64_t>(k) * n + d];
          }
        }
        As[ak][ar] = v;
      }
      {  // B: k bk, column bc (columns fastest across lanes)
        const int bk = idx >> 5, bc = idx & 31;
        const int q = kb + bk, cc = c0 + bc;
        double v = 0.0;
        if (q < K && cc < n) {
          if (MODE == 1) {
            const int d = q > cc ? q - cc : cc - q;
            v = vrow[d];
          } else {
            v = bptr[static_cast<int64_t>(q) * n + cc];
          }
        }
        Bs[bk][bc] = v;
      }
    }
    __syncthreads();
    for (int s = 0; s < 4; ++s) {
      const int kk = s * 4 + (l >> 4);
      double av[2], bv[2];
      for (int i = 0; i < 2; ++i) av[i] = As[kk][i * 16 + (l & 15)];
      for (int j = 0; j < 2; ++j) bv[j] = Bs[kk][j * 16 + (l & 15)];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + i * 16 + (l >> 4) + 4 * v, cc = c0 + j * 16 + (l & 15);
        if (r < n && cc < n) cptr[static_cast<int64_t>(r) * n + cc] = alpha * acc[i][j][v];
      }
}

// j' = (j - grain mean) on grain cells, zero elsewhere, both components
__global__ void __launch_bounds__(256) masked_current_kernel(const double* __restrict__ j,
                                                             const uint8_t* __restrict__ mask, int64_t ncell,
                                                             const double* __restrict__ mean,
                                                             double* __restrict__ jp) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  const bool in = mask[i] != 0;
  jp[i] = in ? j[i] - mean[0] : 0.0;
  jp[ncell + i] = in ? j[ncell + i] - mean[1] : 0.0;
}

// (x - cx) j_y - (y - cy) j_x at every grain cell (grain-cell order)
__global__ void __launch_bounds__(256) torque_kernel(const double* __restrict__ j,
                                                     const int32_t* __restrict__ grain_cells, int64_t ncg,
                                                     int64_t ncell, int nx, double x0, double y0, double h,
                                                     double cx, double cy, double* __restrict__ out) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncg) return;
  const int cell = grain_cells[c];
  const double x = x0 + ((cell % nx) + 0.5) * h - cx, y = y0 + ((cell / nx) + 0.5) * h - cy;
  out[c] = x * j[ncell + cell] - y * j[cell];
}

static inline unsigned nb256(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

void launch_eig_vecpot(int n, int nmodes, const double* jp, const double* vk, const double* lam, double* y,
                       double* aout, double alpha, hipStream_t st) {
  const unsigned t = static_cast<unsigned>((n + 31) / 32);
  hipLaunchKernelGGL(eig_gemm_kernel<1>, dim3(t, t, 2 * nmodes), dim3(64), 0, st, n, nmodes, jp, vk, lam, y, aout,
                     1.0);
  hipLaunchKernelGGL(eig_gemm_kernel<2>, dim3(t, t, 2), dim3(64), 0, st, n, nmodes, jp, vk, lam, y, aout, alpha);
}
void launch_masked_current(const double* j, const uint8_t* mask, int64_t ncell, const double* mean, double* jp,
                           hipStream_t st) {
  if (ncell > 0) hipLaunchKernelGGL(masked_current_kernel, dim3(nb256(ncell)), dim3(256), 0, st, j, mask, ncell, mean, jp);
}
void launch_torque(const double* j, const int32_t* grain_cells, int64_t ncg, int64_t ncell, int nx, double x0,
                   double y0, double h, double cx, double cy, double* out, hipStream_t st) {
  if (ncg > 0)
    hipLaunchKernelGGL(torque_kernel, dim3(nb256(ncg)), dim3(256), 0, st, j, grain_cells, ncg, ncell, nx, x0, y0, h,
                       cx, cy, out);
}

}  // namespace qc
