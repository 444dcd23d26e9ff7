// Weighted join size and its adjoint.
//
// Every row r of table t carries a weight w_t(r); the weighted join size is
// W = sum over result tuples of the product of their rows' weights, which is
// the partition function of Eq. 3 with each table's potential holding the
// summed weights of an entry's rows instead of its row count (Sec. 3.2
// potentials, generalized).  So:
//   forward   cw(e) = sum of w over e's rows; the upward pass of Algorithm 2 in
//             float64: Uw(e) = prod of the children's messages at e,
//             Mw(s) = sum over entries with separator s of cw * Uw,
//             W = sum over root entries of cw * Uw.
//   backward  W is linear in each weight, dW/dw_t(r) = Uw(e(r)) * Dw(e(r))
//             where Dw is the downward message (the conditioning of
//             Algorithms 3-4) computed with cw in place of c:
//             Dw_t(s) = sum over parent entries e' with e'[col] = s of
//             cw(e') * Dw_p(e') * prod of the siblings' messages; Dw = 1 at
//             the root.  This is the adjoint of the forward pass: one
//             downward sweep yields the gradient of every weight.
// Sums over a group run per wavefront (entries of a group are contiguous) and
// one float64 atomic per run; an entry's weights are summed the same way over
// its grouped row positions; downward terms are summed per tile in an LDS
// hash table first.  At unit weights every value is an integer below 2^53,
// so every order of summation gives the exact integer counts.
#include <mutex>
#include <vector>

#include "kernels.h"
#include "plan.h"

using namespace gjh;

struct gj_wstate {
  gj_ctx* ctx = nullptr;
  gj_factors* f = nullptr;
  Arena arena;
  double* cw = nullptr;   // per entry slot: summed weights
  double* Uw = nullptr;   // per entry slot
  double* Mw = nullptr;   // per group slot
  double* Dw = nullptr;   // per group slot
  int32_t* link = nullptr;  // per parent entry, per child (link regions)
  double* W = nullptr;
  std::vector<const void*> w;  // weights (borrowed; must stay valid until backward)
  int dtype = 1;
  explicit gj_wstate(gj_ctx* c) : arena(c) {}
};

namespace {

__device__ __forceinline__ int32_t find_sorted_w(const int32_t* __restrict__ a, int64_t n, int32_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < n && a[lo] == v) ? (int32_t)lo : -1;
}

struct WPtrs {
  const void* w[GJ_MAX_TABLES];  // per table (weighted factors hold one query)
  double* cw;
  double* Uw;
  double* Mw;
  double* Dw;
  int32_t* link;
  double* W;
  int dtype;  // 0 f32, 1 f64
};

__device__ __forceinline__ double wget(const WPtrs& P, int t, int64_t r) {
  return P.dtype ? reinterpret_cast<const double*>(P.w[t])[r] : (double)reinterpret_cast<const float*>(P.w[t])[r];
}

// The entry whose rows hold grouped position i: the last entry starting at
// or before i (entries cover the positions in order, the first at 0).
__device__ __forceinline__ int32_t entry_of_position(const int32_t* __restrict__ estart, int64_t M, int32_t i) {
  int64_t lo = 0, hi = M;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (estart[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  return (int32_t)lo;
}

__device__ __forceinline__ double shfl_up_f64(double v, int off) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)b, off);
  const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(b >> 32), off);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Per entry: summed weights of its rows (cw zeroed beforehand).  One thread
// per grouped row position, so an entry of many rows (a heavy key) is summed
// by many threads: each wave adds up its runs of equal entries (positions are
// in entry order) and the run's last lane adds the run's sum with one atomic.
__global__ void __launch_bounds__(GJ_BLOCK) k_wcount(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                     FPtrs F, WPtrs P) {
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  const int ln = lane_id();
  const int64_t wave0 = base + (threadIdx.x - ln);
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    if (wave0 + r * GJ_BLOCK >= d.n) break;  // wave-uniform
    const int64_t i = base + r * GJ_BLOCK + threadIdx.x;
    int32_t e = -1;
    double v = 0.0;
    if (i < d.n) {
      e = entry_of_position(F.estart + d.off, M, (int32_t)i);
      v = wget(P, w.t, F.perm[d.off + i]);
    }
    const int32_t eprev = __shfl_up(e, 1);
    const bool head = ln == 0 || eprev != e;
    const uint64_t heads = __ballot(head);
    const int sst = 63 - __clzll(heads & (ln == 63 ? ~0ull : ((2ull << ln) - 1)));
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double u = shfl_up_f64(v, off);
      if (ln - off >= sst) v += u;
    }
    const int32_t enext = __shfl_down(e, 1);
    const bool tail = ln == 63 || enext != e;
    if (tail && e >= 0) atomicAdd(&P.cw[d.off + e], v);
  }
}

// Upward step for the tables of one height: Uw, links, and the group sums Mw
// (zeroed beforehand) by one atomic per run of equal groups in a wavefront.
__global__ void __launch_bounds__(GJ_BLOCK) k_wup(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                  FPtrs F, WPtrs P) {
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  if (base >= M) return;
  const int ln = lane_id();
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
    const bool valid = e < M;
    const int64_t se = d.off + e;
    double cu = 0.0;
    int32_t g = -1;
    if (valid) {
      double U = 1.0;
      for (int i = 0; i < d.nchild; ++i) {
        const int ch = d.child[i];
        const TDesc& dc = D[ch];
        const int32_t v = F.ekey[d.key_off + (int64_t)d.child_col[i] * d.n + e];
        const int32_t j = find_sorted_w(F.gval + dc.off, F.cnt[ch * CNT_STRIDE + CNT_G], v);
        P.link[dc.link_off + e] = j;
        U *= j >= 0 ? P.Mw[dc.off + j] : 0.0;
      }
      P.Uw[se] = U;
      cu = P.cw[se] * U;
      g = F.egrp[se];
    }
    // segmented sum over runs of equal g inside the wavefront
    const int32_t gprev = __shfl_up(g, 1, 64);
    uint32_t head = (ln == 0 || gprev != g) ? 1u : 0u;
    double v = cu;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double y = __shfl_up(v, o, 64);
      const uint32_t hy = __shfl_up(head, o, 64);
      if (ln >= o && !head) v += y;
      if (ln >= o) head |= hy;
    }
    const int32_t gnext = __shfl_down(g, 1, 64);
    const bool last = ln == 63 || gnext != g;
    if (valid && last) {
      if (d.is_root)
        atomicAdd(P.W, v);
      else
        atomicAdd(P.Mw + d.off + g, v);
    }
  }
}

#define WDOWN_HASH 2048
// Downward step into the children of the tables in the work list.
__global__ void __launch_bounds__(GJ_BLOCK) k_wdown(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                    FPtrs F, WPtrs P) {
  __shared__ int32_t hkey[WDOWN_HASH];
  __shared__ double hval[WDOWN_HASH];
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  if (base >= M) return;
  for (int ci = 0; ci < d.nchild; ++ci) {
    const TDesc& dt = D[d.child[ci]];
    for (int i = threadIdx.x; i < WDOWN_HASH; i += GJ_BLOCK) {
      hkey[i] = -1;
      hval[i] = 0.0;
    }
    __syncthreads();
    for (int r = 0; r < GJ_ROUNDS; ++r) {
      const int64_t e = base + r * GJ_BLOCK + threadIdx.x;
      if (e >= M) break;
      const int64_t se = d.off + e;
      const int32_t j = P.link[dt.link_off + e];
      if (j < 0) continue;
      const double Dp = d.is_root ? 1.0 : P.Dw[d.off + F.egrp[se]];
      double term = P.cw[se] * Dp;
      for (int i = 0; i < d.nchild; ++i) {
        if (i == ci) continue;
        const TDesc& dc = D[d.child[i]];
        const int32_t jj = P.link[dc.link_off + e];
        term *= jj >= 0 ? P.Mw[dc.off + jj] : 0.0;
      }
      if (term == 0.0) continue;
      const uint32_t h = ((uint32_t)j * 2654435761u) >> 21;
      bool placed = false;
#pragma unroll 1
      for (int p = 0; p < 8 && !placed; ++p) {
        const uint32_t slot = (h + p) & (WDOWN_HASH - 1);
        const int32_t prev = atomicCAS(&hkey[slot], -1, j);
        if (prev == -1 || prev == j) {
          atomicAdd(&hval[slot], term);
          placed = true;
        }
      }
      if (!placed) atomicAdd(P.Dw + dt.off + j, term);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < WDOWN_HASH; i += GJ_BLOCK) {
      const int32_t j = hkey[i];
      if (j >= 0) atomicAdd(P.Dw + dt.off + j, hval[i]);
    }
    __syncthreads();
  }
}

// Per row: gradW * Uw(e) * Dw(e), written in the weight dtype.
struct GPtrs {
  void* g[GJ_MAX_TABLES];
};

// One thread per grouped row position (an entry of many rows is spread over
// many threads).
__global__ void __launch_bounds__(GJ_BLOCK) k_wgrad(const WorkItem* __restrict__ wl, const TDesc* __restrict__ D,
                                                    FPtrs F, WPtrs P, const double* __restrict__ gW, GPtrs grad) {
  const WorkItem w = wl[blockIdx.x];
  const TDesc& d = D[w.t];
  const int64_t M = F.cnt[w.t * CNT_STRIDE + CNT_M];
  const int64_t base = (int64_t)w.tile * GJ_TILE;
  const double g0 = *gW;
  void* gp = grad.g[w.t];
  for (int r = 0; r < GJ_ROUNDS; ++r) {
    const int64_t i = base + r * GJ_BLOCK + threadIdx.x;
    if (i >= d.n) break;
    const int64_t se = d.off + entry_of_position(F.estart + d.off, M, (int32_t)i);
    const double Dv = d.is_root ? 1.0 : P.Dw[d.off + F.egrp[se]];
    const double gv = g0 * P.Uw[se] * Dv;
    const int32_t row = F.perm[d.off + i];
    if (P.dtype)
      reinterpret_cast<double*>(gp)[row] = gv;
    else
      reinterpret_cast<float*>(gp)[row] = (float)gv;
  }
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void fill_f64(hipStream_t s, double* p, int64_t n, double v) {
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>((n + GJ_BLOCK - 1) / GJ_BLOCK, 4096);
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks), dim3(GJ_BLOCK), 0, s, p, n, v);
}

WPtrs wptrs(const gj_wstate* st) {
  WPtrs P{};
  for (size_t t = 0; t < st->w.size(); ++t) P.w[t] = st->w[t];
  P.cw = st->cw;
  P.Uw = st->Uw;
  P.Mw = st->Mw;
  P.Dw = st->Dw;
  P.link = st->link;
  P.W = st->W;
  P.dtype = st->dtype;
  return P;
}

}  // namespace

extern "C" {

gj_status gj_weighted_forward(gj_ctx* ctx, const gj_factors* fc, const void* const* w, int32_t w_dtype, double* d_W,
                              gj_wstate** saved) {
  GJ_SCOPE(ctx);
  if (!ctx || !fc || !w || !d_W || !saved || (w_dtype != 0 && w_dtype != 1)) {
    set_error("gj_weighted_forward: bad argument");
    return GJ_E_INVALID;
  }
  gj_factors* f = const_cast<gj_factors*>(fc);
  const Plan& Pl = f->plan;
  if (Pl.nq != 1) {
    set_error("gj_weighted_forward: factors of a single query expected");
    return GJ_E_INVALID;
  }
  for (int t = 0; t < Pl.nt; ++t)
    if (Pl.ht[t].n > 0 && !w[t]) {
      set_error("gj_weighted_forward: null weights for table %d", t);
      return GJ_E_INVALID;
    }
  gj_wstate* st = new gj_wstate(ctx);
  st->ctx = ctx;
  st->f = f;
  f->refs++;
  st->w.assign(w, w + Pl.nt);
  st->dtype = w_dtype;
  st->cw = st->arena.get_n<double>(Pl.S);
  st->Uw = st->arena.get_n<double>(Pl.S);
  st->Mw = st->arena.get_n<double>(Pl.S);
  st->Dw = st->arena.get_n<double>(Pl.S);
  st->link = st->arena.get_n<int32_t>(Pl.link_slots);
  st->W = st->arena.get_n<double>(1);
  if (!st->cw || !st->Uw || !st->Mw || !st->Dw || !st->link || !st->W) {
    gj_free_wstate(st);
    return GJ_E_OOM;
  }
  hipStream_t s = ctx->stream;
  const WPtrs P = wptrs(st);
  fill_f64(s, st->Mw, Pl.S, 0.0);
  fill_f64(s, st->W, 1, 0.0);
  fill_f64(s, st->cw, Pl.S, 0.0);
  hipLaunchKernelGGL(k_wcount, dim3(std::max(1, Pl.all.n)), dim3(GJ_BLOCK), 0, s, Pl.d_wl + Pl.all.off, Pl.d_desc,
                     f->F, P);
  for (int h = 0; h <= Pl.max_height; ++h) {
    const WL& l = Pl.up[h];
    if (l.n > 0) hipLaunchKernelGGL(k_wup, dim3(l.n), dim3(GJ_BLOCK), 0, s, Pl.d_wl + l.off, Pl.d_desc, f->F, P);
  }
  gj_status stt = check(hipMemcpyAsync(d_W, st->W, 8, hipMemcpyDeviceToDevice, s), "weighted forward");
  if (!stt) stt = check(hipGetLastError(), "weighted forward kernels");
  if (stt) {
    gj_free_wstate(st);
    return stt;
  }
  *saved = st;
  return GJ_OK;
}

gj_status gj_weighted_backward(gj_ctx* ctx, const gj_wstate* stc, const double* d_gradW, void* const* grad_w) {
  GJ_SCOPE(ctx);
  if (!ctx || !stc || !d_gradW || !grad_w) {
    set_error("gj_weighted_backward: bad argument");
    return GJ_E_INVALID;
  }
  gj_wstate* st = const_cast<gj_wstate*>(stc);
  const Plan& Pl = st->f->plan;
  for (int t = 0; t < Pl.nt; ++t)
    if (Pl.ht[t].n > 0 && !grad_w[t]) {
      set_error("gj_weighted_backward: null gradient buffer for table %d", t);
      return GJ_E_INVALID;
    }
  hipStream_t s = ctx->stream;
  const WPtrs P = wptrs(st);
  GPtrs G{};
  for (int t = 0; t < Pl.nt; ++t) G.g[t] = grad_w[t];
  fill_f64(s, st->Dw, Pl.S, 0.0);
  for (int dd = 1; dd <= Pl.max_depth; ++dd) {
    const WL& l = Pl.down[dd];
    if (l.n > 0) hipLaunchKernelGGL(k_wdown, dim3(l.n), dim3(GJ_BLOCK), 0, s, Pl.d_wl + l.off, Pl.d_desc, st->f->F, P);
  }
  if (Pl.all.n > 0)
    hipLaunchKernelGGL(k_wgrad, dim3(Pl.all.n), dim3(GJ_BLOCK), 0, s, Pl.d_wl + Pl.all.off, Pl.d_desc, st->f->F, P,
                       d_gradW, G);
  return check(hipGetLastError(), "weighted backward kernels");
}

void gj_free_wstate(gj_wstate* st) {
  if (!st) return;
  gj_factors* f = st->f;
  st->arena.release();
  delete st;
  if (f) gj_free_factors(f);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The same forward + adjoint with no allocation.  All intermediate state of
// the call (per entry slot cw, Uw; per group slot Mw, Dw; the links; the unit
// incoming gradient) lives in `scratch`, a fixed array every device that runs
// the library holds until the process ends.  Host code never passes the
// array's name to a kernel: the array's device address on each device is
// looked up once with hipGetSymbolAddress and kept per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[GJ_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on ctx's device (looked up on the first call
// made on that device, with the device current).
gj_status scratch_address(gj_ctx* ctx, unsigned char** out) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices) {
    set_error("gj_weighted_grad_noalloc: device %d out of range", ctx->device);
    return GJ_E_INVALID;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    int cur = -1;
    gj_status st = check(hipGetDevice(&cur), "hipGetDevice");
    if (st) return st;
    if (cur != ctx->device && (st = check(hipSetDevice(ctx->device), "hipSetDevice"))) return st;
    void* p = nullptr;
    st = check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
    if (cur != ctx->device) {
      const gj_status st2 = check(hipSetDevice(cur), "hipSetDevice");
      if (!st) st = st2;
    }
    if (st) return st;
    if (!p) {
      set_error("gj_weighted_grad_noalloc: no device address for the scratch array");
      return GJ_E_DEVICE;
    }
    g_scratch_ptr[ctx->device] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[ctx->device]);
  return GJ_OK;
}

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

}  // namespace

extern "C" {

gj_status gj_weighted_grad_noalloc(gj_ctx* ctx, const gj_factors* fc, const void* const* w, int32_t w_dtype,
                                   const double* d_gradW, double* d_W, void* const* grad_w) {
  GJ_SCOPE(ctx);
  if (!ctx || !fc || !w || !d_W || !grad_w || (w_dtype != 0 && w_dtype != 1)) {
    set_error("gj_weighted_grad_noalloc: bad argument");
    return GJ_E_INVALID;
  }
  const gj_factors* f = fc;
  const Plan& Pl = f->plan;
  if (Pl.nq != 1) {
    set_error("gj_weighted_grad_noalloc: factors of a single query expected");
    return GJ_E_INVALID;
  }
  for (int t = 0; t < Pl.nt; ++t)
    if (Pl.ht[t].n > 0 && (!w[t] || !grad_w[t])) {
      set_error("gj_weighted_grad_noalloc: null weights or gradient buffer for table %d", t);
      return GJ_E_INVALID;
    }
  // scratch layout: cw, Uw (entry slots), Mw, Dw (group slots), links, one double
  const int64_t b_slots = align256(Pl.S * (int64_t)sizeof(double));
  const int64_t b_link = align256(Pl.link_slots * (int64_t)sizeof(int32_t));
  const int64_t need = 4 * b_slots + b_link + 256;
  if (need > (int64_t)GJ_NOALLOC_SCRATCH_BYTES) {
    set_error("gj_weighted_grad_noalloc: the query needs %lld bytes of scratch, more than the %lld available "
              "(about %lld rows in all); use gj_weighted_forward / gj_weighted_backward",
              (long long)need, (long long)GJ_NOALLOC_SCRATCH_BYTES,
              (long long)(GJ_NOALLOC_SCRATCH_BYTES / 36));
    return GJ_E_INVALID;
  }
  unsigned char* base = nullptr;
  gj_status st = scratch_address(ctx, &base);
  if (st) return st;
  WPtrs P{};
  for (int t = 0; t < Pl.nt; ++t) P.w[t] = w[t];
  P.cw = reinterpret_cast<double*>(base);
  P.Uw = reinterpret_cast<double*>(base + b_slots);
  P.Mw = reinterpret_cast<double*>(base + 2 * b_slots);
  P.Dw = reinterpret_cast<double*>(base + 3 * b_slots);
  P.link = reinterpret_cast<int32_t*>(base + 4 * b_slots);
  double* one = reinterpret_cast<double*>(base + 4 * b_slots + b_link);
  P.W = d_W;
  P.dtype = w_dtype;
  GPtrs G{};
  for (int t = 0; t < Pl.nt; ++t) G.g[t] = grad_w[t];
  hipStream_t s = ctx->stream;
  // what accumulates starts at zero (fill kernels, no memset: the call may be
  // recorded into a graph)
  fill_f64(s, P.Mw, Pl.S, 0.0);
  fill_f64(s, P.Dw, Pl.S, 0.0);
  fill_f64(s, P.cw, Pl.S, 0.0);
  fill_f64(s, d_W, 1, 0.0);
  if (!d_gradW) {
    fill_f64(s, one, 1, 1.0);
    d_gradW = one;
  }
  if (Pl.all.n > 0)
    hipLaunchKernelGGL(k_wcount, dim3(Pl.all.n), dim3(GJ_BLOCK), 0, s, Pl.d_wl + Pl.all.off, Pl.d_desc, f->F, P);
  for (int h = 0; h <= Pl.max_height; ++h) {
    const WL& l = Pl.up[h];
    if (l.n > 0) hipLaunchKernelGGL(k_wup, dim3(l.n), dim3(GJ_BLOCK), 0, s, Pl.d_wl + l.off, Pl.d_desc, f->F, P);
  }
  for (int dd = 1; dd <= Pl.max_depth; ++dd) {
    const WL& l = Pl.down[dd];
    if (l.n > 0) hipLaunchKernelGGL(k_wdown, dim3(l.n), dim3(GJ_BLOCK), 0, s, Pl.d_wl + l.off, Pl.d_desc, f->F, P);
  }
  if (Pl.all.n > 0)
    hipLaunchKernelGGL(k_wgrad, dim3(Pl.all.n), dim3(GJ_BLOCK), 0, s, Pl.d_wl + Pl.all.off, Pl.d_desc, f->F, P,
                       d_gradW, G);
  return check(hipGetLastError(), "weighted kernels");
}


}  // extern "C"
