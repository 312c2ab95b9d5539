// Warm-start network on gfx950: BF16 matrix-core (MFMA) products with FP32
// accumulation and fused epilogues (bias, GELU, GELU'), loss, bias gradients,
// split-K weight gradients and Adam.  The C ABI is declared in include/mlp.h.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/mlp.h"
#include "../../include/pic.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int NL = MLP_NLAYER;
constexpr int OUTS[NL] = {256, 256, 256, 256, MLP_NOUT};
constexpr int INS[NL] = {MLP_NIN, 256, 256, 256, 256};
constexpr int MAXSPLIT = 16;      // split-K partials of one weight gradient
constexpr int LOSS_BLOCKS = 1024;

__host__ __device__ constexpr int64_t w_off(int l) {
  int64_t k = 0;
  for (int i = 0; i < l; ++i) k += (int64_t)OUTS[i] * INS[i] + OUTS[i];
  return k;
}
__host__ __device__ constexpr int64_t b_off(int l) { return w_off(l) + (int64_t)OUTS[l] * INS[l]; }
static_assert(w_off(NL) == MLP_NPARAM, "parameter count");

// ---------------------------------------------------------------- GELU (exact erf)
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_prime(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// ---------------------------------------------------------------- tiled product
// C[m][n] = sum_k A(m, k) B(k, n), A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn]
// (bfloat16), FP32 sums on the matrix cores.  A block of 4 waves owns a 64 x 64
// tile; each wave a 32 x 32 quarter as 2 x 2 products of v_mfma_f32_16x16x32_bf16,
// k taken TK at a time through LDS and 32 at a time through the matrix cores.
// blockIdx.z selects a K range of kchunk (split-K partials).
enum { EPI_STORE = 0, EPI_HIDDEN = 1, EPI_OUT = 2, EPI_BWD = 3 };

struct GemmArgs {
  const __bf16 *A;
  int64_t sam, sak;
  const __bf16 *B;
  int64_t sbk, sbn;
  int M, N, K, kchunk;
  float *C;            // STORE: partials [split][M][N]; HIDDEN: pre-activations; OUT: outputs; BWD: dz
  __bf16 *C16;         // HIDDEN: activations; BWD: dz in bfloat16
  const float *bias;   // HIDDEN, OUT
  const float *zin;    // BWD: pre-activations of the layer below
};

constexpr int TM = 64, TN = 64, TK = 32, TKP = TK + 8;   // LDS rows padded by 16 bytes
constexpr int TV = TM * TK / 8 / 256;                      // 16-byte vectors per thread and tile

// The 64 x TK tile T[r][k] = X(r0 + r, k0 + k), X(r, k) = P[r sr + k sk], zero
// outside r < R, k < ke.  Along whichever index is contiguous in memory each
// thread moves 8 elements with one 16-byte load when they are in range and
// aligned (k contiguous: activations and weights of the forward pass and of the
// input gradient; r contiguous: the output gradients of the weight gradient).
__device__ __forceinline__ void load_tile(__bf16 (*T)[TKP], const __bf16 *P, int64_t sr, int64_t sk, int r0, int R,
                                          int k0, int ke, int t) {
  const __bf16 zero = (__bf16)0.0f;
  constexpr int KV = TK / 8;                     // vectors along k per row
  for (int v = 0; v < TV; ++v) {
    const int q = v * 256 + t;                   // vector index in the tile
    if (sk == 1) {
      const int lr = q / KV, lk = (q % KV) * 8;
      const int r = r0 + lr, k = k0 + lk;
      const __bf16 *src = P + (int64_t)r * sr + k;
      if (r < R && k + 8 <= ke && ((uintptr_t)src & 15) == 0) {
        *reinterpret_cast<bf16x8 *>(&T[lr][lk]) = *reinterpret_cast<const bf16x8 *>(src);
      } else {
        for (int i = 0; i < 8; ++i) T[lr][lk + i] = (r < R && k + i < ke) ? src[i] : zero;
      }
    } else if (sr == 1) {
      const int lk = q / (TM / 8), lr = (q % (TM / 8)) * 8;
      const int r = r0 + lr, k = k0 + lk;
      const __bf16 *src = P + r + (int64_t)k * sk;
      if (k < ke && r + 8 <= R && ((uintptr_t)src & 15) == 0) {
        const bf16x8 x = *reinterpret_cast<const bf16x8 *>(src);
        for (int i = 0; i < 8; ++i) T[lr + i][lk] = x[i];
      } else {
        for (int i = 0; i < 8; ++i) T[lr + i][lk] = (k < ke && r + i < R) ? src[i] : zero;
      }
    } else {
      const int lr = q / KV, lk = (q % KV) * 8;
      const int r = r0 + lr;
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + lk + i;
        T[lr][lk + i] = (r < R && k < ke) ? P[(int64_t)r * sr + (int64_t)k * sk] : zero;
      }
    }
  }
}

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __align__(16) __bf16 As[TM][TKP];
  __shared__ __align__(16) __bf16 Bs[TN][TKP];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kb = blockIdx.z * g.kchunk, ke = min(g.K, kb + g.kchunk);
  floatx4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = kb; k0 < ke; k0 += TK) {
    load_tile(As, g.A, g.sam, g.sak, m0, g.M, k0, ke, t);
    load_tile(Bs, g.B, g.sbn, g.sbk, n0, g.N, k0, ke, t);
    __syncthreads();
    const int kq = 8 * (lane >> 4), rr = lane & 15;
    const int ksub = min(TK, ke - k0);             // products of 32 k values in order, as many as the tile holds
    for (int kk = 0; kk < ksub; kk += 32) {
      bf16x8 a[2], b[2];
      for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(&As[wr * 32 + i * 16 + rr][kk + kq]);
      for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wc * 32 + j * 16 + rr][kk + kq]);
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // result layout of a 16 x 16 product: lane l holds rows 4 (l / 16) + v, column l % 16
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wr * 32 + i * 16 + 4 * (lane >> 4) + v;
        const int n = n0 + wc * 32 + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        const float x = acc[i][j][v];
        const int64_t o = (int64_t)m * g.N + n;
        if (EPI == EPI_STORE) {
          g.C[(int64_t)blockIdx.z * g.M * g.N + o] = x;
        } else if (EPI == EPI_HIDDEN) {
          const float z = x + g.bias[n];
          g.C[o] = z;
          g.C16[o] = (__bf16)gelu(z);
        } else if (EPI == EPI_OUT) {
          g.C[o] = x + g.bias[n];
        } else {
          const float dz = x * gelu_prime(g.zin[o]);
          g.C[o] = dz;
          g.C16[o] = (__bf16)dz;
        }
      }
}

// ---------------------------------------------------------------- small kernels
__global__ void k_to_bf16(const float *x, __bf16 *y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (__bf16)x[i];
}

// d loss / d y = 2 (y - t) / (6 B) and per-block sums of (y - t)^2
__global__ __launch_bounds__(256) void k_loss(const float *y, const float *t, float *dz, __bf16 *dz16, float *part,
                                              int64_t n, float scale) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float d = y[i] - t[i];
    s += d * d;
    const float g = scale * d;
    dz[i] = g;
    dz16[i] = (__bf16)g;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_loss_sum(const float *part, int nb, float inv_n, float *loss) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * inv_n;
}

// bias gradient: column sums of dz [rows][cols], one block per column, fixed order
__global__ __launch_bounds__(256) void k_colsum(const float *dz, int64_t rows, int cols, float *out) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.0f;
  for (int64_t r = threadIdx.x; r < rows; r += 256) s += dz[r * cols + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

__global__ void k_sum_splits(const float *part, int nsplit, int64_t n, float *out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * n + i];
    out[i] = s;
  }
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, __bf16 *p16, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    p16[i] = (__bf16)pi;
  }
}

// ---------------------------------------------------------------- workspace
struct Layout {
  size_t total = 0;
  size_t p32, p16, g, m, v, xb, z[NL - 1], act[NL - 1], y, dz32[2], dz16[2], part, lossp, loss;
  size_t take(size_t bytes) {
    const size_t o = total;
    total += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

Layout make_layout(int64_t B) {
  Layout L;
  const size_t P = MLP_NPARAM;
  L.p32 = L.take(4 * P);
  L.p16 = L.take(2 * P);
  L.g = L.take(4 * P);
  L.m = L.take(4 * P);
  L.v = L.take(4 * P);
  L.xb = L.take(2 * (size_t)B * MLP_NIN);
  for (int l = 0; l < NL - 1; ++l) {
    L.z[l] = L.take(4 * (size_t)B * MLP_NHID);
    L.act[l] = L.take(2 * (size_t)B * MLP_NHID);
  }
  L.y = L.take(4 * (size_t)B * MLP_NOUT);
  for (int k = 0; k < 2; ++k) {
    L.dz32[k] = L.take(4 * (size_t)B * MLP_NHID);
    L.dz16[k] = L.take(2 * (size_t)B * MLP_NHID);
  }
  L.part = L.take(4 * (size_t)MAXSPLIT * MLP_NHID * MLP_NHID);
  L.lossp = L.take(4 * LOSS_BLOCKS);
  L.loss = L.take(4);
  return L;
}

std::string g_err;

// Activations of mlp_forward_static: one file-scope array per device (each GPU
// the library runs on holds its copy until the process ends).  Layout for up to
// MLP_STATIC_MAX_BATCH samples: the bfloat16 input, one FP32 pre-activation
// buffer and two bfloat16 activation buffers used in turn by the hidden layers.
constexpr size_t ST_XB = 0;
constexpr size_t ST_Z = ((size_t)MLP_STATIC_MAX_BATCH * MLP_NIN * 2 + 255) & ~(size_t)255;
constexpr size_t ST_ACT0 = ST_Z + (size_t)MLP_STATIC_MAX_BATCH * MLP_NHID * 4;
constexpr size_t ST_ACT1 = ST_ACT0 + (size_t)MLP_STATIC_MAX_BATCH * MLP_NHID * 2;
constexpr size_t ST_BYTES = ST_ACT1 + (size_t)MLP_STATIC_MAX_BATCH * MLP_NHID * 2;
static_assert(ST_BYTES == MLP_STATIC_SCRATCH_BYTES, "scratch size stated in mlp.h");

static __device__ __align__(256) unsigned char scratch[ST_BYTES];

// device address of `scratch` per device, looked up once with that device current
constexpr int MAX_DEVICES = 64;
unsigned char *g_scratch_dev[MAX_DEVICES] = {};
std::mutex g_scratch_mu;

hipError_t scratch_address(int dev, unsigned char **out) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = (unsigned char *)p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

}  // namespace

struct mlp_handle {
  int32_t max_batch = 0;
  unsigned char *scratch = nullptr;   // this device's activation array of mlp_forward_static
  Layout L;
  unsigned char *ws = nullptr;
  hipStream_t stream = nullptr;
  int64_t adam_step = 0;
  std::string err;
  template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

namespace {

int fail(mlp_handle *h, int code, const std::string &m) {
  if (h) h->err = m;
  else g_err = m;
  return code;
}

#define MHIP(h, expr)                                                                                \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) return fail((h), PIC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <int EPI>
hipError_t gemm(const GemmArgs &g, int split, hipStream_t st) {
  const dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM, split);
  hipLaunchKernelGGL((k_gemm<EPI>), grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

int grid_of(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

// Forward pass over `batch` samples of x (FP32, device) into y.  xb: the
// bfloat16 input; z[l], act[l]: pre-activation (FP32) and activation (bfloat16)
// of hidden layer l (the buffers of different layers may coincide when only the
// output is wanted and act[l] != act[l - 1]).
struct FwdBufs { __bf16 *xb; float *z[NL - 1]; __bf16 *act[NL - 1]; };

int forward_into(mlp_handle *h, int32_t batch, const float *x, const FwdBufs &b, float *y) {
  hipStream_t st = h->stream;
  const int64_t nx = (int64_t)batch * MLP_NIN;
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_of(nx)), dim3(256), 0, st, x, b.xb, nx);
  MHIP(h, hipGetLastError());
  for (int l = 0; l < NL; ++l) {
    GemmArgs g{};
    g.A = l == 0 ? b.xb : b.act[l - 1];
    g.sam = INS[l];
    g.sak = 1;
    g.B = h->at<__bf16>(h->L.p16) + w_off(l);       // B(k, n) = W[n][k]
    g.sbk = 1;
    g.sbn = INS[l];
    g.M = batch;
    g.N = OUTS[l];
    g.K = INS[l];
    g.kchunk = INS[l];
    g.bias = h->at<float>(h->L.p32) + b_off(l);
    if (l + 1 < NL) {
      g.C = b.z[l];
      g.C16 = b.act[l];
      MHIP(h, gemm<EPI_HIDDEN>(g, 1, st));
    } else {
      g.C = y;
      MHIP(h, gemm<EPI_OUT>(g, 1, st));
    }
  }
  return PIC_OK;
}

// forward pass with every activation kept in the workspace (training)
int run_forward(mlp_handle *h, int32_t batch, const float *x) {
  const Layout &L = h->L;
  FwdBufs b;
  b.xb = h->at<__bf16>(L.xb);
  for (int l = 0; l < NL - 1; ++l) {
    b.z[l] = h->at<float>(L.z[l]);
    b.act[l] = h->at<__bf16>(L.act[l]);
  }
  return forward_into(h, batch, x, b, h->at<float>(L.y));
}

int refresh_bf16(mlp_handle *h) {
  const int64_t n = MLP_NPARAM;
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_of(n)), dim3(256), 0, h->stream, h->at<float>(h->L.p32),
                     h->at<__bf16>(h->L.p16), n);
  MHIP(h, hipGetLastError());
  return PIC_OK;
}

}  // namespace

extern "C" {

int mlp_query(int32_t max_batch, uint64_t *bytes) {
  if (max_batch < 1 || max_batch > (1 << 20) || !bytes) return fail(nullptr, PIC_EINVAL, "max_batch must be in [1, 2^20]");
  *bytes = make_layout(max_batch).total;
  return PIC_OK;
}

int mlp_create(int32_t max_batch, void *workspace, uint64_t bytes, void *stream, mlp_handle **out) {
  uint64_t need = 0;
  int rc = mlp_query(max_batch, &need);
  if (rc != PIC_OK) return rc;
  if (!workspace || !out) return fail(nullptr, PIC_EINVAL, "null workspace or handle pointer");
  if (bytes < need) return fail(nullptr, PIC_EINVAL, "workspace smaller than mlp_query reported");
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(nullptr, PIC_ENODEVICE, "no HIP device");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, PIC_ENODEVICE, std::string("device is ") + prop.gcnArchName + ", kernels are for gfx950");
  unsigned char *scr = nullptr;
  const hipError_t es = scratch_address(dev, &scr);
  if (es != hipSuccess)
    return fail(nullptr, PIC_EHIP, std::string("mlp_create: hipGetSymbolAddress(scratch): ") + hipGetErrorString(es));
  mlp_handle *h = new mlp_handle();
  h->max_batch = max_batch;
  h->scratch = scr;
  h->L = make_layout(max_batch);
  h->ws = (unsigned char *)workspace;
  h->stream = (hipStream_t)stream;
  const hipError_t e = hipMemsetAsync(h->ws, 0, h->L.total, h->stream);
  if (e != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) {
    delete h;
    return fail(nullptr, PIC_EHIP, "mlp_create: clearing the workspace failed");
  }
  *out = h;
  return PIC_OK;
}

int mlp_destroy(mlp_handle *h) {
  if (!h) return PIC_EINVAL;
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return PIC_OK;
}

int mlp_set_params(mlp_handle *h, const float *p) {
  if (!h || !p) return fail(h, PIC_EINVAL, "null argument");
  MHIP(h, hipMemcpyAsync(h->at<float>(h->L.p32), p, 4 * (size_t)MLP_NPARAM, hipMemcpyHostToDevice, h->stream));
  const int rc = refresh_bf16(h);
  if (rc != PIC_OK) return rc;
  MHIP(h, hipStreamSynchronize(h->stream));
  return PIC_OK;
}

int mlp_get_params(mlp_handle *h, float *p) {
  if (!h || !p) return fail(h, PIC_EINVAL, "null argument");
  MHIP(h, hipStreamSynchronize(h->stream));
  MHIP(h, hipMemcpy(p, h->at<float>(h->L.p32), 4 * (size_t)MLP_NPARAM, hipMemcpyDeviceToHost));
  return PIC_OK;
}

int mlp_forward(mlp_handle *h, int32_t batch, const float *x, float *y) {
  if (!h || !x || !y || batch < 1 || batch > h->max_batch) return fail(h, PIC_EINVAL, "need 1 <= batch <= max_batch and non-null x, y");
  const int rc = run_forward(h, batch, x);
  if (rc != PIC_OK) return rc;
  MHIP(h, hipMemcpyAsync(y, h->at<float>(h->L.y), 4 * (size_t)batch * MLP_NOUT, hipMemcpyDeviceToDevice, h->stream));
  return PIC_OK;
}

int mlp_forward_static(mlp_handle *h, int32_t batch, const float *x, float *y) {
  if (!h || !x || !y) return fail(h, PIC_EINVAL, "null handle, x or y");
  if (batch < 1 || batch > MLP_STATIC_MAX_BATCH)
    return fail(h, PIC_EINVAL, "mlp_forward_static: batch must be in [1, " + std::to_string(MLP_STATIC_MAX_BATCH) +
                                   "] (the size of the library's static activation array)");
  FwdBufs b;
  b.xb = reinterpret_cast<__bf16 *>(h->scratch + ST_XB);
  for (int l = 0; l < NL - 1; ++l) {
    b.z[l] = reinterpret_cast<float *>(h->scratch + ST_Z);
    b.act[l] = reinterpret_cast<__bf16 *>(h->scratch + ((l & 1) ? ST_ACT1 : ST_ACT0));
  }
  return forward_into(h, batch, x, b, y);
}

int mlp_backward(mlp_handle *h, int32_t batch, const float *x, const float *t, float *loss_host) {
  if (!h || !x || !t || batch < 1 || batch > h->max_batch) return fail(h, PIC_EINVAL, "need 1 <= batch <= max_batch and non-null x, t");
  int rc = run_forward(h, batch, x);
  if (rc != PIC_OK) return rc;
  const Layout &L = h->L;
  hipStream_t st = h->stream;
  const int64_t ny = (int64_t)batch * MLP_NOUT;
  const int lb = (int)std::min<int64_t>(LOSS_BLOCKS, (ny + 255) / 256);
  int cur = 0;                                  // dz buffers of the layer being differentiated
  hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, st, h->at<float>(L.y), t, h->at<float>(L.dz32[cur]),
                     h->at<__bf16>(L.dz16[cur]), h->at<float>(L.lossp), ny, 2.0f / (float)ny);
  MHIP(h, hipGetLastError());
  hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, st, h->at<float>(L.lossp), lb, 1.0f / (float)ny,
                     h->at<float>(L.loss));
  MHIP(h, hipGetLastError());
  const int split = (int)std::min<int64_t>(MAXSPLIT, std::max<int64_t>(1, batch / 1024));
  const int kchunk = ((batch + split - 1) / split + 31) / 32 * 32;
  for (int l = NL - 1; l >= 0; --l) {
    const int out = OUTS[l], in = INS[l];
    const __bf16 *a_in = l == 0 ? h->at<__bf16>(L.xb) : h->at<__bf16>(L.act[l - 1]);
    // dW[o][i] = sum_b dz[b][o] a_in[b][i]
    GemmArgs gw{};
    gw.A = h->at<__bf16>(L.dz16[cur]);
    gw.sam = 1;
    gw.sak = out;
    gw.B = a_in;
    gw.sbk = in;
    gw.sbn = 1;
    gw.M = out;
    gw.N = in;
    gw.K = batch;
    gw.kchunk = kchunk;
    gw.C = h->at<float>(L.part);
    MHIP(h, gemm<EPI_STORE>(gw, split, st));
    const int64_t nw = (int64_t)out * in;
    hipLaunchKernelGGL(k_sum_splits, dim3(grid_of(nw)), dim3(256), 0, st, h->at<float>(L.part), split, nw,
                       h->at<float>(L.g) + w_off(l));
    MHIP(h, hipGetLastError());
    hipLaunchKernelGGL(k_colsum, dim3(out), dim3(256), 0, st, h->at<float>(L.dz32[cur]), (int64_t)batch, out,
                       h->at<float>(L.g) + b_off(l));
    MHIP(h, hipGetLastError());
    if (l == 0) break;
    // dz of the layer below: (dz W)[b][i] GELU'(z[b][i])
    GemmArgs gd{};
    gd.A = h->at<__bf16>(L.dz16[cur]);
    gd.sam = out;
    gd.sak = 1;
    gd.B = h->at<__bf16>(L.p16) + w_off(l);     // B(k, n) = W[k][n]
    gd.sbk = in;
    gd.sbn = 1;
    gd.M = batch;
    gd.N = in;
    gd.K = out;
    gd.kchunk = out;
    gd.C = h->at<float>(L.dz32[1 - cur]);
    gd.C16 = h->at<__bf16>(L.dz16[1 - cur]);
    gd.zin = h->at<float>(L.z[l - 1]);
    MHIP(h, gemm<EPI_BWD>(gd, 1, st));
    cur = 1 - cur;
  }
  if (loss_host) {
    MHIP(h, hipMemcpyAsync(loss_host, h->at<float>(L.loss), 4, hipMemcpyDeviceToHost, st));
    MHIP(h, hipStreamSynchronize(st));
  }
  return PIC_OK;
}

int mlp_get_grads(mlp_handle *h, float *g) {
  if (!h || !g) return fail(h, PIC_EINVAL, "null argument");
  MHIP(h, hipStreamSynchronize(h->stream));
  MHIP(h, hipMemcpy(g, h->at<float>(h->L.g), 4 * (size_t)MLP_NPARAM, hipMemcpyDeviceToHost));
  return PIC_OK;
}

int mlp_adam(mlp_handle *h, float lr, float b1, float b2, float eps) {
  if (!h) return PIC_EINVAL;
  if (!(lr >= 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps > 0.0f))
    return fail(h, PIC_EINVAL, "need lr >= 0, 0 <= beta < 1, eps > 0");
  const int64_t k = ++h->adam_step;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)k)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)k)));
  const Layout &L = h->L;
  const int64_t n = MLP_NPARAM;
  hipLaunchKernelGGL(k_adam, dim3(grid_of(n)), dim3(256), 0, h->stream, h->at<float>(L.p32), h->at<float>(L.g),
                     h->at<float>(L.m), h->at<float>(L.v), h->at<__bf16>(L.p16), n, lr, b1, b2, eps, c1, c2);
  MHIP(h, hipGetLastError());
  return PIC_OK;
}

const char *mlp_last_error(const mlp_handle *h) { return h ? h->err.c_str() : g_err.c_str(); }

}  // extern "C"
