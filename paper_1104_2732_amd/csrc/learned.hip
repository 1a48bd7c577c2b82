// Learned bracket proposal: synthetic mixture arrays, array sketches (features), a small
// network with its forward, backward and Adam kernels, and the single-array bracket kernel
// that feeds the selection's two-point pass 0.
//
// This extends the method; nothing here decides a result.  The selection keeps a proposed
// end only where the counts of its own pass 0 prove it (Section 4's bracket invariant
// #(x <= yL) < k <= #(x < yR)), so a poor network costs passes, never exactness.
//
// Precision: the generator and the features follow definitions made of integer and
// correctly rounded double operations (identical bits on any conforming implementation);
// the network runs in float, every sum in a fixed order (the results are deterministic).
#include "cps_device.h"
#include "cps_kernels.h"

namespace cps {

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11:
// ten rounds of two 32x32->64 multiplications with the published multipliers, the key
// bumped by the published Weyl constants between rounds.

struct U4 {
  uint32_t x, y, z, w;
};

__device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// ------------------------------------------------------------------ exp from basic operations
// 2^floor(t) * P(f ln 2), t = z log2(e), f = t - floor(t), P the degree-14 Taylor
// polynomial of e^g in Horner form with coefficients 1/j! formed by successive division.

template <int J> struct InvFact {
  static constexpr double v = InvFact<J - 1>::v / (double)J;
};
template <> struct InvFact<0> {
  static constexpr double v = 1.0;
};
// (..((c14 g + c13) g + c12) ..) g + c0
template <int J> __device__ inline double horner_exp(double g) {
  if constexpr (J == 14) return InvFact<14>::v;
  else return horner_exp<J + 1>(g) * g + InvFact<J>::v;
}

__device__ inline double exp_basic(double z) {
  const double t = z * 1.4426950408889634;
  const double kf = floor(t);
  const double g = (t - kf) * 0.6931471805599453;
  return ldexp(horner_exp<0>(g), (int)kf);
}

// ------------------------------------------------------------------ mixture arrays

enum : int32_t { MIX_GAUSS = 0, MIX_LOGNORMAL = 1, MIX_UNIFORM = 2 };

struct Mixture {
  double cum[4], p1[4], p2[4];
  int32_t types[4];
  int32_t ncomp;
  int64_t k;
};

__device__ inline Mixture mixture_params(uint64_t seed, uint32_t id, int64_t n) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  uint32_t w[20];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const U4 r = philox4x32_10(U4{0u, 0u, id, (uint32_t)(4 + j)}, k0, k1);
    w[4 * j + 0] = r.x;
    w[4 * j + 1] = r.y;
    w[4 * j + 2] = r.z;
    w[4 * j + 3] = r.w;
  }
  Mixture m;
  m.ncomp = 1 + (int32_t)(w[0] >> 30);
  uint64_t q[4], tot = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    q[j] = 1 + (uint64_t)(w[13 + j] >> 8);
    if (j < m.ncomp) tot += q[j];
  }
  const double totd = (double)tot;
  uint64_t acc = 0;
  const double ln10 = 2.302585092994046;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool on = j < m.ncomp;
    acc += on ? q[j] : 0;
    const int32_t ty = (int32_t)(((uint64_t)w[1 + j] * 3u) >> 32);
    const double ua = (double)w[5 + j] * 0x1p-32;
    const double ub = (double)w[9 + j] * 0x1p-32;
    const double wide = -100.0 + 200.0 * ua;               // Gaussian mean, uniform start
    const double sd_g = exp_basic((-2.0 + 3.0 * ub) * ln10);
    const double len_u = exp_basic((-2.0 + 4.0 * ub) * ln10);
    const double p1 = ty == MIX_LOGNORMAL ? -2.0 + 4.0 * ua : wide;
    const double p2 = ty == MIX_GAUSS ? sd_g : (ty == MIX_LOGNORMAL ? 0.25 + 1.25 * ub : len_u);
    m.cum[j] = on ? (double)acc / totd : 1.0;
    m.types[j] = on ? ty : 0;
    m.p1[j] = on ? p1 : 0.0;
    m.p2[j] = on ? p2 : 0.0;
  }
  const uint64_t u64 = ((uint64_t)w[17] << 32) | w[18];
  m.k = 1 + (int64_t)__umul64hi(u64, (uint64_t)n);
  return m;
}

__device__ inline float mixture_value(const Mixture &m, uint64_t i, uint32_t id, uint32_t k0,
                                      uint32_t k1) {
  const uint32_t lo = (uint32_t)i, hi = (uint32_t)(i >> 32);
  double g = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const U4 r = philox4x32_10(U4{lo, hi, id, (uint32_t)j}, k0, k1);
    g = g + (double)(r.x >> 8) * 0x1p-24;
    g = g + (double)(r.y >> 8) * 0x1p-24;
    g = g + (double)(r.z >> 8) * 0x1p-24;
    g = g + (double)(r.w >> 8) * 0x1p-24;
  }
  g = g - 6.0;
  const U4 r3 = philox4x32_10(U4{lo, hi, id, 3u}, k0, k1);
  const double uc = (double)r3.x * 0x1p-32;
  const double uu = (double)r3.y * 0x1p-32;
  int comp = 0;
#pragma unroll
  for (int j = 0; j < 3; ++j) comp += uc >= m.cum[j] ? 1 : 0;
  if (comp > m.ncomp - 1) comp = m.ncomp - 1;
  const double p1 = m.p1[comp], p2 = m.p2[comp];
  const int32_t t = m.types[comp];
  double v;
  if (t == MIX_GAUSS) v = p1 + p2 * g;
  else if (t == MIX_LOGNORMAL) v = exp_basic(p1 + p2 * g);
  else v = p1 + p2 * uu;
  return (float)v;
}

constexpr int kGenBlock = 256;
constexpr int kGenPerThread = 16;

__global__ __launch_bounds__(kGenBlock) void mixture_gen_kernel(uint64_t seed, int64_t first_id,
                                                                int64_t n, float *out,
                                                                int64_t *ks) {
  // the array's mixture, formed once per workgroup and read from LDS
  __shared__ Mixture m;
  const int64_t a = blockIdx.y;
  const uint32_t id = (uint32_t)(first_id + a);
  if (threadIdx.x == 0) {
    m = mixture_params(seed, id, n);
    if (ks && blockIdx.x == 0) ks[a] = m.k;
  }
  __syncthreads();
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  CPS_GLOBAL float *o = (CPS_GLOBAL float *)(out + a * n);
  for (int64_t i = (int64_t)blockIdx.x * kGenBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kGenBlock)
    o[i] = mixture_value(m, (uint64_t)i, id, k0, k1);
}

hipError_t launch_mixture_gen(uint64_t seed, int64_t first_id, int64_t count, int64_t n,
                              float *out, int64_t *ks, hipStream_t stream) {
  int64_t bx = (n + (int64_t)kGenBlock * kGenPerThread - 1) / ((int64_t)kGenBlock * kGenPerThread);
  if (bx < 1) bx = 1;
  for (int64_t c0 = 0; c0 < count; c0 += 65535) {
    const int64_t c = count - c0 < 65535 ? count - c0 : 65535;
    mixture_gen_kernel<<<dim3((unsigned)bx, (unsigned)c), dim3(kGenBlock), 0, stream>>>(
        seed, first_id + c0, n, out + c0 * n, ks ? ks + c0 : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ features

constexpr int kSample = 4096;
constexpr int kBins = 64;
constexpr int kIn = kBins + 3;
constexpr int kHid = 64;
constexpr int kOut = 2;
constexpr int kParams = kHid * kIn + kHid + kHid * kHid + kHid + kOut * kHid + kOut;
static_assert(kParams == CPS_MLP_PARAMS, "parameter count");
constexpr int kOffW1 = 0, kOffB1 = kHid * kIn, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
              kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kOut * kHid;
constexpr int kFeatBlock = 256;

struct FeatShared {
  double v[kSample];
  uint32_t hist[kBins];
  double rmin[kFeatBlock / kWave], rmax[kFeatBlock / kWave];
  int rbad[kFeatBlock / kWave];
  double lo, hi;
  int bad;
};

// The 67 features of one array, computed by one workgroup of kFeatBlock threads into f
// (any memory); lo/hi/valid are set in every thread.
template <typename T>
__device__ void array_features(const T *x, int64_t n, int64_t k, FeatShared &fs, float *f,
                               double &lo_out, double &hi_out, int &valid_out) {
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  const int64_t S = n < kSample ? n : kSample;
  const int64_t stride = n / S;
  double mn = __builtin_inf(), mx = -__builtin_inf();
  int bad = 0;
  // all of this thread's strided loads in flight at once (each is its own cache line)
  constexpr int PER = kSample / kFeatBlock;
  double vv[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t i = tid + (int64_t)j * kFeatBlock;
    vv[j] = i < S ? (double)x[i * stride] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t i = tid + (int64_t)j * kFeatBlock;
    if (i < S) {
      const double v = vv[j];
      fs.v[i] = v;
      if (!__builtin_isfinite(v)) bad = 1;
      else {
        mn = fmin(mn, v);
        mx = fmax(mx, v);
      }
    }
  }
  mn = wave_min(mn);
  mx = wave_max(mx);
  const int wbad = __builtin_amdgcn_ballot_w64(bad != 0) != 0 ? 1 : 0;
  if (lane == 0) {
    fs.rmin[wv] = mn;
    fs.rmax[wv] = mx;
    fs.rbad[wv] = wbad;
  }
  if (tid < kBins) fs.hist[tid] = 0u;
  __syncthreads();
  if (tid == 0) {
    double a = fs.rmin[0], b = fs.rmax[0];
    int c = fs.rbad[0];
    for (int w = 1; w < kFeatBlock / kWave; ++w) {
      a = fmin(a, fs.rmin[w]);
      b = fmax(b, fs.rmax[w]);
      c |= fs.rbad[w];
    }
    fs.lo = a + 0.0;  // a zero extreme is +0
    fs.hi = b + 0.0;
    fs.bad = c;
  }
  __syncthreads();
  const double lo = fs.lo, hi = fs.hi;
  const bool valid = fs.bad == 0;
  if (valid) {
    const double span = hi - lo;
    for (int64_t i = tid; i < S; i += kFeatBlock) {
      int b = 0;
      if (hi > lo) {
        const double q = (64.0 * (fs.v[i] - lo)) / span;
        b = (int)floor(q);
        if (b > kBins - 1) b = kBins - 1;
      }
      atomicAdd(&fs.hist[b], 1u);
    }
  }
  __syncthreads();
  if (tid < kIn) {
    float fv = 0.0f;
    if (valid) {
      if (tid < kBins) {
        uint32_t cum = 0;  // the fraction of the sample in bins 0..tid
        for (int b = 0; b <= tid; ++b) cum += fs.hist[b];
        fv = (float)((double)cum / (double)S);
      } else if (tid == kBins) {
        fv = (float)(lo / (1.0 + fabs(lo)));
      } else if (tid == kBins + 1) {
        fv = (float)(hi / (1.0 + fabs(hi)));
      } else {
        fv = (float)((double)k / (double)n);
      }
    }
    f[tid] = fv;
  }
  lo_out = valid ? lo : 0.0;
  hi_out = valid ? hi : 0.0;
  valid_out = valid ? 1 : 0;
}

template <typename T>
__global__ __launch_bounds__(kFeatBlock) void features_kernel(const T *const *ptrs,
                                                              const int64_t *sizes,
                                                              const int64_t *ks, float *feat,
                                                              double *range, int32_t *valid) {
  __shared__ FeatShared fs;
  const int64_t a = blockIdx.x;
  const T *x = ptrs[a];
  const int64_t n = sizes[a], k = ks[a];
  float *f = feat + a * kIn;
  if (!x || n < 1 || k < 1 || k > n || ((uintptr_t)x % sizeof(T)) != 0) {
    if (threadIdx.x < kIn) f[threadIdx.x] = 0.0f;
    if (threadIdx.x == 0) {
      range[2 * a] = range[2 * a + 1] = 0.0;
      valid[a] = 0;
    }
    return;
  }
  double lo, hi;
  int ok;
  array_features<T>(x, n, k, fs, f, lo, hi, ok);
  if (threadIdx.x == 0) {
    range[2 * a] = lo;
    range[2 * a + 1] = hi;
    valid[a] = ok;
  }
}

template <typename T>
hipError_t launch_features(const T *const *ptrs, const int64_t *sizes, const int64_t *ks,
                           int64_t count, float *feat, double *range, int32_t *valid,
                           hipStream_t stream) {
  for (int64_t c0 = 0; c0 < count; c0 += (int64_t)1 << 30) {
    const int64_t c = count - c0 < ((int64_t)1 << 30) ? count - c0 : ((int64_t)1 << 30);
    features_kernel<T><<<dim3((unsigned)c), dim3(kFeatBlock), 0, stream>>>(
        ptrs + c0, sizes + c0, ks + c0, feat + c0 * kIn, range + 2 * c0, valid + c0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ the network

constexpr int kEPW = 32;  // examples per workgroup
constexpr int kMlpBlock = 256;
constexpr int kHS = kHid + 1;  // padded row stride of the activation tiles

// Activations of R rows: inputs, pre-activations of both hidden layers, outputs.
template <int R> struct MlpTile {
  float X[R][kIn];
  float Z1[R][kHS];
  float Z2[R][kHS];
  float O[R][kOut];
};

struct MlpGradShared {
  MlpTile<kEPW> t;
  float D2[kEPW][kHS];
  float D1[kEPW][kHS];
  float dO[kEPW][kOut];
  float lossv[kEPW];
};

__device__ inline float relu(float v) { return v > 0.0f ? v : 0.0f; }

// Forward pass of rows 0..nr-1 of sh.X: pre-activations Z1, Z2 and outputs O.  Every sum
// runs over its input index in increasing order with separately rounded products, then
// adds the bias.
template <int R>
__device__ void mlp_forward_rows(const float *__restrict__ P, MlpTile<R> &sh, int nr) {
  const int tid = threadIdx.x, j = tid % kHid, eg = tid / kHid;
  constexpr int NG = kMlpBlock / kHid;
  {
    float w[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) w[i] = P[kOffW1 + j * kIn + i];
    const float b = P[kOffB1 + j];
    for (int e = eg; e < nr; e += NG) {
      float s = 0.0f;
#pragma unroll
      for (int i = 0; i < kIn; ++i) s = s + w[i] * sh.X[e][i];
      sh.Z1[e][j] = s + b;
    }
  }
  __syncthreads();
  {
    float w[kHid];
#pragma unroll
    for (int i = 0; i < kHid; ++i) w[i] = P[kOffW2 + j * kHid + i];
    const float b = P[kOffB2 + j];
    for (int e = eg; e < nr; e += NG) {
      float s = 0.0f;
#pragma unroll
      for (int i = 0; i < kHid; ++i) s = s + w[i] * relu(sh.Z1[e][i]);
      sh.Z2[e][j] = s + b;
    }
  }
  __syncthreads();
  if (tid < kOut * nr) {
    const int e = tid / kOut, o = tid % kOut;
    float s = 0.0f;
    for (int i = 0; i < kHid; ++i) s = s + P[kOffW3 + o * kHid + i] * relu(sh.Z2[e][i]);
    sh.O[e][o] = s + P[kOffB3 + o];
  }
  __syncthreads();
}

__device__ inline void load_rows(const float *__restrict__ feat, int64_t r0, int nr,
                                 MlpTile<kEPW> &sh) {
  for (int q = threadIdx.x; q < nr * kIn; q += kMlpBlock) sh.X[q / kIn][q % kIn] = feat[r0 * kIn + q];
  __syncthreads();
}

__global__ __launch_bounds__(kMlpBlock) void mlp_forward_kernel(const float *__restrict__ P,
                                                                const float *__restrict__ feat,
                                                                int64_t count,
                                                                float *__restrict__ out) {
  __shared__ MlpTile<kEPW> sh;
  const int64_t r0 = (int64_t)blockIdx.x * kEPW;
  const int nr = (int)(count - r0 < kEPW ? count - r0 : kEPW);
  load_rows(feat, r0, nr, sh);
  mlp_forward_rows<kEPW>(P, sh, nr);
  if (threadIdx.x < kOut * nr) {
    const int e = threadIdx.x / kOut, o = threadIdx.x % kOut;
    out[(r0 + e) * kOut + o] = sh.O[e][o];
  }
}

constexpr float kCSq = 100.0f, kCCov = 1.0f, kCW = 0.02f, kLogWMin = -20.0f, kLogWMax = 4.0f;

// Partial loss and gradient of this workgroup's rows (the mean's 1/B already applied);
// sums over the workgroup's examples run in increasing example order.
__global__ __launch_bounds__(kMlpBlock) void mlp_grad_kernel(const float *__restrict__ P,
                                                             const float *__restrict__ feat,
                                                             const float *__restrict__ ustar,
                                                             int64_t count,
                                                             float *__restrict__ part,
                                                             float *__restrict__ part_loss) {
  __shared__ MlpGradShared sh;
  MlpTile<kEPW> &tl = sh.t;
  const int tid = threadIdx.x, lane = tid % kHid, eg = tid / kHid;
  constexpr int NG = kMlpBlock / kHid;
  const int64_t r0 = (int64_t)blockIdx.x * kEPW;
  const int nr = (int)(count - r0 < kEPW ? count - r0 : kEPW);
  const float invB = 1.0f / (float)count;
  float *G = part + (int64_t)blockIdx.x * kParams;
  load_rows(feat, r0, nr, tl);
  mlp_forward_rows<kEPW>(P, tl, nr);
  // d loss / d outputs
  if (tid < nr) {
    const int e = tid;
    const float u = tl.O[e][0], sv = tl.O[e][1];
    const float d = u - ustar[r0 + e];
    const bool in_clamp = sv > kLogWMin && sv < kLogWMax;
    const float w = expf(fminf(fmaxf(sv, kLogWMin), kLogWMax));
    const float ad = fabsf(d);
    const bool out_cov = ad > w;
    const float sgn = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
    sh.lossv[e] = (kCSq * d * d + kCCov * (out_cov ? ad - w : 0.0f) + kCW * w) * invB;
    sh.dO[e][0] = (2.0f * kCSq * d + (out_cov ? kCCov * sgn : 0.0f)) * invB;
    sh.dO[e][1] = in_clamp ? ((out_cov ? -kCCov : 0.0f) + kCW) * w * invB : 0.0f;
  }
  __syncthreads();
  // layer 3: dZ2, dW3, db3
  {
    const float w0 = P[kOffW3 + lane], w1 = P[kOffW3 + kHid + lane];
    for (int e = eg; e < nr; e += NG) {
      const float da = sh.dO[e][0] * w0 + sh.dO[e][1] * w1;
      sh.D2[e][lane] = tl.Z2[e][lane] > 0.0f ? da : 0.0f;
    }
  }
  if (tid < kOut * kHid) {
    const int o = tid / kHid, j = tid % kHid;
    float s = 0.0f;
    for (int e = 0; e < nr; ++e) s = s + sh.dO[e][o] * relu(tl.Z2[e][j]);
    G[kOffW3 + o * kHid + j] = s;
  }
  if (tid < kOut) {
    float s = 0.0f;
    for (int e = 0; e < nr; ++e) s = s + sh.dO[e][tid];
    G[kOffB3 + tid] = s;
  }
  if (tid == 0) {
    float s = 0.0f;
    for (int e = 0; e < nr; ++e) s = s + sh.lossv[e];
    part_loss[blockIdx.x] = s;
  }
  __syncthreads();
  // layer 2: dZ1 = (dZ2 W2) masked, dW2, db2
  {
    float wc[kHid];  // column `lane` of W2
#pragma unroll
    for (int j = 0; j < kHid; ++j) wc[j] = P[kOffW2 + j * kHid + lane];
    for (int e = eg; e < nr; e += NG) {
      float s = 0.0f;
#pragma unroll
      for (int j = 0; j < kHid; ++j) s = s + sh.D2[e][j] * wc[j];
      sh.D1[e][lane] = tl.Z1[e][lane] > 0.0f ? s : 0.0f;
    }
  }
  for (int r = 0; r < kHid / NG; ++r) {
    const int j = eg + NG * r, i = lane;
    float s = 0.0f;
    for (int e = 0; e < nr; ++e) s = s + sh.D2[e][j] * relu(tl.Z1[e][i]);
    G[kOffW2 + j * kHid + i] = s;
  }
  if (tid < kHid) {
    float s = 0.0f;
    for (int e = 0; e < nr; ++e) s = s + sh.D2[e][tid];
    G[kOffB2 + tid] = s;
  }
  __syncthreads();
  // layer 1: dW1, db1
  for (int q = tid; q < kHid * kIn; q += kMlpBlock) {
    const int j = q / kIn, i = q % kIn;
    float s = 0.0f;
    for (int e = 0; e < nr; ++e) s = s + sh.D1[e][j] * tl.X[e][i];
    G[kOffW1 + q] = s;
  }
  if (tid < kHid) {
    float s = 0.0f;
    for (int e = 0; e < nr; ++e) s = s + sh.D1[e][tid];
    G[kOffB1 + tid] = s;
  }
}

// Sum of the workgroups' partials, each parameter in increasing workgroup order.
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float *__restrict__ part, int nwg,
                                                         const float *__restrict__ part_loss,
                                                         float *__restrict__ grad,
                                                         float *__restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < kParams) {
    float s = 0.0f;
    for (int w = 0; w < nwg; ++w) s = s + part[(int64_t)w * kParams + p];
    grad[p] = s;
  }
  if (loss && p == 0) {
    float s = 0.0f;
    for (int w = 0; w < nwg; ++w) s = s + part_loss[w];
    *loss = s;
  }
}

hipError_t launch_mlp_forward(const float *P, const float *feat, int64_t count, float *out,
                              hipStream_t stream) {
  const int64_t nwg = (count + kEPW - 1) / kEPW;
  mlp_forward_kernel<<<dim3((unsigned)nwg), dim3(kMlpBlock), 0, stream>>>(P, feat, count, out);
  return hipGetLastError();
}

size_t mlp_grad_workspace(int64_t count) {
  const int64_t nwg = (count + kEPW - 1) / kEPW;
  return (size_t)nwg * (kParams + 1) * sizeof(float) + 256;
}

hipError_t launch_mlp_loss_grad(const float *P, const float *feat, const float *ustar,
                                int64_t count, float *grad, float *loss, float *ws,
                                hipStream_t stream) {
  const int64_t nwg = (count + kEPW - 1) / kEPW;
  float *part = ws;
  float *part_loss = ws + nwg * kParams;
  mlp_grad_kernel<<<dim3((unsigned)nwg), dim3(kMlpBlock), 0, stream>>>(P, feat, ustar, count, part,
                                                                       part_loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  mlp_reduce_kernel<<<dim3((kParams + 255) / 256), dim3(256), 0, stream>>>(part, (int)nwg, part_loss,
                                                                          grad, loss);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float *__restrict__ P,
                                                       const float *__restrict__ g,
                                                       float *__restrict__ m,
                                                       float *__restrict__ v, float lr, float b1,
                                                       float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kParams) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.0f - b1) * gp;
  const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  P[p] = P[p] - lr * (mp * c1) / (sqrtf(vp * c2) + eps);
}

hipError_t launch_mlp_adam(float *P, const float *g, float *m, float *v, int64_t step, float lr,
                           float b1, float b2, float eps, hipStream_t stream) {
  // bias corrections 1 / (1 - b^step), formed in double on the host
  const float c1 = (float)(1.0 / (1.0 - pow((double)b1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)b2, (double)step)));
  mlp_adam_kernel<<<dim3((kParams + 255) / 256), dim3(256), 0, stream>>>(P, g, m, v, lr, b1, b2, eps,
                                                                        c1, c2);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void mlp_init_kernel(uint64_t seed, float *__restrict__ P) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kParams) return;
  float bound = 0.0f;
  if (p < kOffB1) bound = sqrtf(6.0f / (float)kIn);
  else if (p >= kOffW2 && p < kOffB2) bound = sqrtf(6.0f / (float)kHid);
  else if (p >= kOffW3 && p < kOffB3) bound = 0.01f * sqrtf(6.0f / (float)kHid);
  const U4 r = philox4x32_10(U4{(uint32_t)p, 0u, 0u, 0xC0FFEEu}, (uint32_t)seed,
                             (uint32_t)(seed >> 32));
  const float u = (float)(r.x >> 8) * 0x1p-24f;
  float val = (2.0f * u - 1.0f) * bound;
  if (p == kOffB3) val = 0.0f;  // start at the histogram's position
  if (p == kOffB3 + 1) val = logf(0.05f);
  P[p] = val;
}

hipError_t launch_mlp_init(uint64_t seed, float *P, hipStream_t stream) {
  mlp_init_kernel<<<dim3((kParams + 255) / 256), dim3(256), 0, stream>>>(seed, P);
  return hipGetLastError();
}

// ------------------------------------------------------------------ proposal of one array

// The histogram's own estimate of the rank's position in the sample range: where the
// cumulative features cross the k/n feature, linear inside the crossing bin.  The network
// predicts the offset from it.
__device__ inline double hist_position(const float *f) {
  const double p = (double)f[kBins + 2];
  int b = 0;
  while (b < kBins - 1 && (double)f[b] < p) ++b;
  const double prev = b > 0 ? (double)f[b - 1] : 0.0;
  const double fb = (double)f[b];
  if (!(fb > prev)) return ((double)b + 0.5) / (double)kBins;
  return ((double)b + (p - prev) / (fb - prev)) / (double)kBins;
}

__device__ inline void proposal_from_outputs(float u, float s, double h, double lo, double hi,
                                             bool valid, double &a, double &b, bool &use) {
  const double span = hi - lo;
  const double sc = fmin(fmax((double)s, (double)kLogWMin), (double)kLogWMax);
  const double y0 = lo + span * (h + (double)u);
  const double w = span * exp(sc);
  a = y0 - w;
  b = y0 + w;
  use = valid && a < b && __builtin_isfinite(a) && __builtin_isfinite(b);
}

template <typename T>
__global__ __launch_bounds__(kMlpBlock) void learned_bracket_kernel(const T *x, int64_t n, int64_t k,
                                                                    const float *__restrict__ P,
                                                                    uint64_t *zero_hist,
                                                                    double *bracket) {
  static_assert(kMlpBlock == kFeatBlock, "one workgroup computes features and network");
  __shared__ FeatShared fs;
  __shared__ MlpTile<1> sh;
  // the counters the selection's pass 0 fills with the proposal's interior start at zero
  if (zero_hist)
    for (int i = threadIdx.x; i < kHistMaxBins; i += kMlpBlock) zero_hist[i] = 0;
  double lo, hi;
  int ok;
  array_features<T>(x, n, k, fs, &sh.X[0][0], lo, hi, ok);
  __syncthreads();
  mlp_forward_rows<1>(P, sh, 1);
  if (threadIdx.x == 0) {
    double a, b;
    bool use;
    proposal_from_outputs(sh.O[0][0], sh.O[0][1], hist_position(&sh.X[0][0]), lo, hi, ok != 0,
                          a, b, use);
    bracket[0] = use ? a : 0.0;
    bracket[1] = use ? b : 0.0;
    bracket[2] = use ? 1.0 : 0.0;
  }
}

template <typename T>
hipError_t launch_learned_bracket(const T *x, int64_t n, int64_t k, const float *P,
                                  uint64_t *zero_hist, double *bracket, hipStream_t stream) {
  learned_bracket_kernel<T><<<dim3(1), dim3(kMlpBlock), 0, stream>>>(x, n, k, P, zero_hist, bracket);
  return hipGetLastError();
}

// ------------------------------------------------------------------ sample-quantile proposal
// The non-learned baseline of the proposal: the same fixed-stride sample, and the bracket
// between its order statistics z standard deviations of the sample rank (binomial,
// sqrt(S p (1 - p)) + 1) below and above the expected rank S k / n.  The two order
// statistics are selected, not sorted for: the sample sits in LDS and the workgroup's radix
// select (8-bit digits of the ordered keys) finds each wanted rank.

constexpr int kSortBlock = 1024;

template <typename T>
__global__ __launch_bounds__(kSortBlock) void sample_bracket_kernel(const T *x, int64_t n,
                                                                   int64_t k, double z,
                                                                   uint64_t *zero_hist,
                                                                   double *bracket) {
  constexpr int PER = kSample / kSortBlock;
  __shared__ double sv[kSample];
  __shared__ uint32_t hist[256];
  __shared__ int64_t misc[4];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (zero_hist)
    for (int i = tid; i < kHistMaxBins; i += kSortBlock) zero_hist[i] = 0;
  const int64_t S = n < kSample ? n : kSample;
  const int64_t stride = n / S;
  if (tid == 0) bad = 0;
  __syncthreads();
  double vv[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {  // the strided loads all in flight
    const int i = tid + j * kSortBlock;
    vv[j] = i < S ? (double)x[i * stride] : 0.0;
  }
  bool nf = false;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = tid + j * kSortBlock;
    if (i < S) {
      nf = nf || !__builtin_isfinite(vv[j]);
      sv[i] = vv[j];
    }
  }
  if (nf) bad = 1;
  __syncthreads();
  if (bad) {
    if (tid == 0) bracket[0] = bracket[1] = bracket[2] = 0.0;
    return;
  }
  const double pr = (double)k / (double)n;
  const double c = pr * (double)S;
  const double sd = sqrt((double)S * pr * (1.0 - pr)) + 1.0;
  const int64_t want[2] = {(int64_t)floor(c - z * sd) - 1, (int64_t)ceil(c + z * sd)};  // 0-based
  double got[2] = {-__builtin_inf(), __builtin_inf()};
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    if (want[w] < 0 || want[w] > S - 1) continue;  // (uniform) an open end
    uint64_t key;
    int64_t below, eq;
    block_radix_select<double, kSortBlock>(sv, S, false, 0.0, 0.0, want[w] + 1, hist, misc, key,
                                           below, eq);
    got[w] = unkey64(key);
  }
  if (tid == 0) {
    bracket[0] = got[0];
    bracket[1] = got[1];
    bracket[2] = 1.0;
  }
}

template <typename T>
hipError_t launch_sample_bracket(const T *x, int64_t n, int64_t k, double z, uint64_t *zero_hist,
                                 double *bracket, hipStream_t stream) {
  sample_bracket_kernel<T><<<dim3(1), dim3(kSortBlock), 0, stream>>>(x, n, k, z, zero_hist, bracket);
  return hipGetLastError();
}

template hipError_t launch_sample_bracket<float>(const float *, int64_t, int64_t, double, uint64_t *,
                                                 double *, hipStream_t);
template hipError_t launch_sample_bracket<double>(const double *, int64_t, int64_t, double, uint64_t *,
                                                  double *, hipStream_t);

// ------------------------------------------------------------------ training helpers

__global__ void batch_descriptor_kernel(const float *base, int64_t n, int64_t count,
                                        const float **ptrs, int64_t *sizes) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < count;
       a += (int64_t)gridDim.x * blockDim.x) {
    ptrs[a] = base + a * n;
    sizes[a] = n;
  }
}

// Labels (x_(k) - lo) / (hi - lo) - h with h the histogram position, 0 where the sample
// was constant or invalid.
__global__ void label_kernel(const cps_result *res, const float *feat, const double *range,
                             const int32_t *valid, int64_t count, float *ustar) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < count;
       a += (int64_t)gridDim.x * blockDim.x) {
    const double lo = range[2 * a], hi = range[2 * a + 1];
    float u = 0.0f;
    if (valid[a] && res[a].status == 0 && hi > lo)
      u = (float)((res[a].value - lo) / (hi - lo) - hist_position(feat + a * kIn));
    ustar[a] = u;
  }
}

// Coverage of held-out arrays: acc[0] += #(a < x_(k) < b), acc[1] += sum of 2 w / (hi - lo),
// acc[2] += #valid (one workgroup, in a fixed order).
__global__ __launch_bounds__(256) void holdout_kernel(const float *out, const float *feat,
                                                      const double *range, const int32_t *valid,
                                                      const cps_result *res, int64_t count,
                                                      double *acc) {
  __shared__ double s0[256], s1[256], s2[256];
  double c = 0, wsum = 0, nv = 0;
  for (int64_t e = threadIdx.x; e < count; e += 256) {
    if (!valid[e] || res[e].status != 0) continue;
    double a, b;
    bool use;
    proposal_from_outputs(out[2 * e], out[2 * e + 1], hist_position(feat + e * kIn), range[2 * e],
                          range[2 * e + 1], true, a, b, use);
    const double v = res[e].value, span = range[2 * e + 1] - range[2 * e];
    nv += 1;
    if (use && a < v && v < b) c += 1;
    if (span > 0) wsum += (b - a) / span;
  }
  s0[threadIdx.x] = c;
  s1[threadIdx.x] = wsum;
  s2[threadIdx.x] = nv;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0, t1 = 0, t2 = 0;
    for (int i = 0; i < 256; ++i) {
      t0 += s0[i];
      t1 += s1[i];
      t2 += s2[i];
    }
    acc[0] += t0;
    acc[1] += t1;
    acc[2] += t2;
  }
}

hipError_t launch_batch_descriptors(const float *base, int64_t n, int64_t count, const float **ptrs,
                                    int64_t *sizes, hipStream_t stream) {
  batch_descriptor_kernel<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream>>>(
      base, n, count, ptrs, sizes);
  return hipGetLastError();
}

hipError_t launch_labels(const cps_result *res, const float *feat, const double *range,
                         const int32_t *valid, int64_t count, float *ustar, hipStream_t stream) {
  label_kernel<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream>>>(res, feat, range,
                                                                               valid, count, ustar);
  return hipGetLastError();
}

hipError_t launch_holdout(const float *out, const float *feat, const double *range,
                          const int32_t *valid, const cps_result *res, int64_t count, double *acc,
                          hipStream_t stream) {
  holdout_kernel<<<dim3(1), dim3(256), 0, stream>>>(out, feat, range, valid, res, count, acc);
  return hipGetLastError();
}

template hipError_t launch_features<float>(const float *const *, const int64_t *, const int64_t *,
                                           int64_t, float *, double *, int32_t *, hipStream_t);
template hipError_t launch_features<double>(const double *const *, const int64_t *,
                                            const int64_t *, int64_t, float *, double *, int32_t *,
                                            hipStream_t);
template hipError_t launch_learned_bracket<float>(const float *, int64_t, int64_t, const float *,
                                                  uint64_t *, double *, hipStream_t);
template hipError_t launch_learned_bracket<double>(const double *, int64_t, int64_t, const float *,
                                                   uint64_t *, double *, hipStream_t);

}  // namespace cps
