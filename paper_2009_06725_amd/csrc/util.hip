// Device-wide scan and adjacency-list construction (integer setup work).
#include "internal.hpp"

namespace scvs {

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

hipEvent_t Profiler::get() {
  if (used == pool.size()) {
    hipEvent_t e;
    SCVS_HIP(hipEventCreate(&e));
    pool.push_back(e);
  }
  return pool[used++];
}

void Profiler::resolve() {
  if (pending.empty() && corrections.empty()) return;
  if (!pending.empty()) SCVS_HIP(hipEventSynchronize(pending.back().b));
  for (auto& pd : pending) {
    float ms = 0.0f;
    SCVS_HIP(hipEventElapsedTime(&ms, pd.a, pd.b));
    auto it = std::find_if(stats.begin(), stats.end(), [&](const auto& kv) { return kv.first == pd.name; });
    if (it == stats.end()) {
      stats.push_back({pd.name, Stat{}});
      it = stats.end() - 1;
    }
    it->second.launches += pd.count;
    it->second.ms += ms;
    it->second.bytes += pd.bytes;
  }
  for (auto& c : corrections)
    for (auto& kv : stats)
      if (kv.first == c.first) kv.second.bytes += c.second;
  corrections.clear();
  pending.clear();
  used = 0;
}

Profiler::~Profiler() {
  for (auto e : pool) (void)hipEventDestroy(e);
}

ProfScope::ProfScope(Profiler* p, hipStream_t s, const char* name, double bytes, int count) : p_(p), s_(s) {
  if (!p_ || !p_->on || capturing(s)) {
    p_ = nullptr;
    return;
  }
  hipEvent_t a = p_->get(), b = p_->get();
  SCVS_HIP(hipEventRecord(a, s));
  p_->pending.push_back({name, a, b, bytes, count});
  idx_ = p_->pending.size() - 1;
}

ProfScope::~ProfScope() {
  if (p_) (void)hipEventRecord(p_->pending[idx_].b, s_);
}

namespace {

constexpr int SCAN_BS = 256;
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_IPT;

template <class In>
__global__ void __launch_bounds__(SCAN_BS) k_scan_tile(const In* __restrict__ in, int64_t n,
                                                       int64_t* __restrict__ out,
                                                       int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[SCAN_BS];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)t * SCAN_IPT;
  int64_t v[SCAN_IPT];
  int64_t tsum = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    v[i] = (base + i < n) ? (int64_t)in[base + i] : 0;
    tsum += v[i];
  }
  sh[t] = tsum;
  __syncthreads();
  for (int off = 1; off < SCAN_BS; off <<= 1) {
    int64_t add = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int64_t run = sh[t] - tsum;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (t == SCAN_BS - 1) bsum[blockIdx.x] = sh[t];
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ boff) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += boff[i / SCAN_TILE];
}

template <class In>
__global__ void k_scan_total(const In* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
  out[n] = (n > 0) ? out[n - 1] + (int64_t)in[n - 1] : 0;
}

template <class In>
void scan_rec(const In* in, int64_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  DBuf<int64_t> bsum, boff;
  bsum.alloc(nb);
  k_scan_tile<In><<<nb, SCAN_BS, 0, s>>>(in, n, out, bsum);
  SCVS_HIP(hipGetLastError());
  if (nb > 1) {
    boff.alloc(nb + 1);
    scan_rec<int64_t>(bsum.p, boff.p, nb, s);
    k_scan_add<<<(n + 255) / 256, 256, 0, s>>>(out, n, boff);
    SCVS_HIP(hipGetLastError());
  }
  SCVS_HIP(hipStreamSynchronize(s));  // temporaries are freed on return
}

template <class In>
int64_t scan_total(const In* in, int64_t* out, int64_t n, hipStream_t s) {
  scan_rec<In>(in, out, n, s);
  k_scan_total<In><<<1, 1, 0, s>>>(in, n, out);
  SCVS_HIP(hipGetLastError());
  int64_t total = 0;
  download(&total, out + n, 1, s);
  return total;
}

__global__ void k_adj_count(const int32_t* __restrict__ ids, int64_t nids, int32_t* __restrict__ cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nids) atomicAdd(&cnt[ids[i]], 1);
}

__global__ void k_adj_fill(const int32_t* __restrict__ ids, int64_t nids, int nper,
                           const int64_t* __restrict__ ptr, int32_t* __restrict__ cursor,
                           int32_t* __restrict__ list) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nids) {
    int32_t t = ids[i];
    int32_t pos = atomicAdd(&cursor[t], 1);
    list[ptr[t] + pos] = (int32_t)(i / nper);
  }
}

// Insertion sort of each (short) list; makes the fill order irrelevant.
__global__ void k_adj_sort(const int64_t* __restrict__ ptr, int64_t ntarget, int32_t* __restrict__ list) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntarget) return;
  int64_t b = ptr[t], e = ptr[t + 1];
  for (int64_t i = b + 1; i < e; ++i) {
    int32_t key = list[i];
    int64_t j = i - 1;
    while (j >= b && list[j] > key) {
      list[j + 1] = list[j];
      --j;
    }
    list[j + 1] = key;
  }
}

}  // namespace

int64_t exclusive_scan(const int64_t* counts, int64_t* out, int64_t n, hipStream_t s) {
  return scan_total<int64_t>(counts, out, n, s);
}
int64_t exclusive_scan32(const int32_t* counts, int64_t* out, int64_t n, hipStream_t s) {
  return scan_total<int32_t>(counts, out, n, s);
}

void build_adjacency(const int32_t* ids, int64_t nitems, int nper, int64_t ntarget,
                     DBuf<int64_t>& ptr, DBuf<int32_t>& list, hipStream_t s) {
  int64_t nids = nitems * nper;
  DBuf<int32_t> cnt;
  cnt.alloc(ntarget);
  cnt.zero(s);
  if (nids) {
    k_adj_count<<<(nids + 255) / 256, 256, 0, s>>>(ids, nids, cnt);
    SCVS_HIP(hipGetLastError());
  }
  ptr.alloc(ntarget + 1);
  int64_t total = exclusive_scan32(cnt, ptr, ntarget, s);
  list.alloc(total);
  cnt.zero(s);
  if (nids) {
    k_adj_fill<<<(nids + 255) / 256, 256, 0, s>>>(ids, nids, nper, ptr, cnt, list);
    SCVS_HIP(hipGetLastError());
  }
  if (ntarget) {
    k_adj_sort<<<(ntarget + 255) / 256, 256, 0, s>>>(ptr, ntarget, list);
    SCVS_HIP(hipGetLastError());
  }
  SCVS_HIP(hipStreamSynchronize(s));
}

}  // namespace scvs
