// Cluster tree, device arenas and the launch executor.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "hodlr.h"

// Workspace of acr_solve_noalloc: one copy per GPU, held until the process
// ends.  Host code never passes this name to a kernel (on the host it is only
// a stand-in); it uses the device address that noalloc_scratch() obtains with
// hipGetSymbolAddress.
static __device__ __align__(256) char scratch[ACR_NOALLOC_SCRATCH_BYTES];

namespace acr {

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory) throw Failure(ST_OOM, std::string(what) + ": out of device memory");
  throw Failure(ST_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T> size_t HMat<T>::words(const Tree& tr) const {
  if (kind == DIAG) return tr.M;
  if (kind != HODLR) return 0;
  size_t w = 0;
  for (int s = 0; s < (1 << tr.L); ++s) w += (size_t)tr.sz[tr.L][s] * tr.sz[tr.L][s];
  for (int d = 0; d < tr.L; ++d)
    for (int s = 0; s < (2 << d); ++s) {
      const auto& b = blk[Tree::bid(d, s)];
      w += (size_t)b.k * (tr.sz[d + 1][s] + tr.sz[d + 1][s ^ 1]);
    }
  return w;
}
template struct HMat<float>;
template struct HMat<double>;

// ---------------------------------------------------------------- arena
void* Arena::get(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  while (ci_ < chunks_.size()) {
    if (off_ + bytes <= chunks_[ci_].second) {
      void* p = chunks_[ci_].first + off_;
      off_ += bytes;
      return p;
    }
    if (fixed_) break;
    ++ci_;
    off_ = 0;
  }
  if (fixed_) {
    char msg[160];
    std::snprintf(msg, sizeof(msg), "workspace exceeds the fixed no-allocation scratch of %zu bytes",
                  chunks_.empty() ? size_t(0) : chunks_[0].second);
    throw Failure(ST_INVALID, msg);
  }
  const size_t csz = std::max(chunk_, bytes);
  char* p = static_cast<char*>(ex_->dev_alloc(csz));
  chunks_.push_back({p, csz});
  ci_ = chunks_.size() - 1;
  off_ = bytes;
  return p;
}

void Arena::init_fixed(void* base, size_t bytes) {
  chunks_.assign(1, {static_cast<char*>(base), bytes});
  chunk_ = 0;
  ci_ = off_ = 0;
  fixed_ = true;
}

void Arena::free_all() {
  if (fixed_) {
    chunks_.clear();
    ci_ = off_ = 0;
    return;
  }
  for (auto& c : chunks_) ex_->dev_free(c.first);
  chunks_.clear();
  ci_ = off_ = 0;
}

size_t Arena::used() const {
  size_t u = 0;
  for (size_t i = 0; i < ci_ && i < chunks_.size(); ++i) u += chunks_[i].second;
  return u + off_;
}

size_t Arena::reserved() const {
  size_t u = 0;
  for (auto& c : chunks_) u += c.second;
  return u;
}

// ---------------------------------------------------------------- timing table
namespace {
std::mutex g_time_mu;
bool g_timing = false;
int g_timing_level = 0;
struct TimeAcc { long launches = 0; double ms = 0, flops = 0, bytes = 0; };
std::map<std::string, TimeAcc>& time_table() {
  static std::map<std::string, TimeAcc> t;
  return t;
}
constexpr size_t kCounters = 1 << 16;
}  // namespace

void timing_enable(int level) {
  std::lock_guard<std::mutex> lk(g_time_mu);
  if (level > 0) time_table().clear();   // a new measurement starts; disabling keeps the table
  g_timing = level > 0;
  g_timing_level = level > 0 ? level : 0;
}
bool timing_enabled() { return g_timing; }
bool solve_timing_enabled() { return g_timing_level >= 2; }

int timing_report(acr_kernel_time_t* out, int cap) {
  std::lock_guard<std::mutex> lk(g_time_mu);
  int n = 0;
  for (auto& kv : time_table()) {
    if (out && n < cap) {
      acr_kernel_time_t& o = out[n];
      std::memset(&o, 0, sizeof(o));
      std::strncpy(o.name, kv.first.c_str(), sizeof(o.name) - 1);
      o.launches = kv.second.launches;
      o.total_ms = kv.second.ms;
      o.flops = kv.second.flops;
      o.bytes = kv.second.bytes;
    }
    ++n;
  }
  return n;
}

unsigned long long* Exec::counter_slot() {
  if (!d_counters_) {
    d_counters_ = static_cast<unsigned long long*>(dev_alloc(kCounters * sizeof(unsigned long long)));
    hip_check(hipMemsetAsync(d_counters_, 0, kCounters * sizeof(unsigned long long), stream), "hipMemsetAsync(ctr)");
  }
  if (counter_cursor_ >= kCounters) {
    sync();
    hip_check(hipMemsetAsync(d_counters_, 0, kCounters * sizeof(unsigned long long), stream), "hipMemsetAsync(ctr)");
    counter_cursor_ = 0;
  }
  return d_counters_ + counter_cursor_++;
}

void Exec::resolve_timings() {
  if (pending_.empty()) return;
  std::vector<unsigned long long> ctr;
  if (d_counters_ && counter_cursor_ > 0) {
    ctr.resize(counter_cursor_);
    hip_check(hipMemcpy(ctr.data(), d_counters_, ctr.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost),
              "hipMemcpy(counters)");
  }
  std::lock_guard<std::mutex> lk(g_time_mu);
  for (auto& p : pending_) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    double fl = p.w.flops, by = p.w.bytes;
    if (p.w.counter && d_counters_) {
      const size_t i = p.w.counter - d_counters_;
      const double c = i < ctr.size() ? (double)ctr[i] : 0.0;
      fl += c * p.w.flops_per_count;
      by += c * p.w.bytes_per_count;
    }
    TimeAcc& a = time_table()[p.w.cls ? p.w.cls : "other"];
    a.launches += 1;
    a.ms += ms;
    a.flops += fl;
    a.bytes += by;
    event_pool_.push_back(p.a);
    event_pool_.push_back(p.b);
  }
  pending_.clear();
  if (d_counters_ && counter_cursor_ > 0) {
    hip_check(hipMemsetAsync(d_counters_, 0, counter_cursor_ * sizeof(unsigned long long), stream),
              "hipMemsetAsync(ctr)");
    counter_cursor_ = 0;
  }
}

// ---------------------------------------------------------------- exec
namespace {
std::mutex g_reg_mu;
std::map<uintptr_t, size_t>& registry() {
  static std::map<uintptr_t, size_t> r;
  return r;
}
void reg_add(void* p, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  registry()[(uintptr_t)p] = bytes;
}
size_t reg_del(void* p) {
  std::lock_guard<std::mutex> lk(g_reg_mu);
  auto it = registry().find((uintptr_t)p);
  if (it == registry().end()) return 0;
  const size_t b = it->second;
  registry().erase(it);
  return b;
}

// Device buffers the library released (default allocator only), kept per
// (device, size) for reuse by later requests of the same size: a factorisation
// allocates its arenas in equal chunks, and hipMalloc / hipFree of such chunks
// synchronise the device and, after many factorisations in one process, took
// up to 0.3 s each.  acr_release_cached_memory() returns them to the runtime;
// an allocation that fails does the same and tries once more.
std::mutex g_pool_mu;
std::map<std::pair<int, size_t>, std::vector<void*>>& chunk_pool() {
  static std::map<std::pair<int, size_t>, std::vector<void*>> p;
  return p;
}
bool pool_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("ACR_NO_POOL");
    return !(e && e[0] == '1');
  }();
  return on;
}
void* pool_take(int dev, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = chunk_pool().find({dev, bytes});
  if (it == chunk_pool().end() || it->second.empty()) return nullptr;
  void* p = it->second.back();
  it->second.pop_back();
  return p;
}
void pool_put(int dev, void* p, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  chunk_pool()[{dev, bytes}].push_back(p);
}
size_t pool_release() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  size_t n = 0;
  for (auto& kv : chunk_pool())
    for (void* p : kv.second) {
      (void)hipFree(p);
      n += kv.first.second;
    }
  chunk_pool().clear();
  return n;
}
}  // namespace

size_t release_cached_memory() { return pool_release(); }

namespace {
struct DeviceScratch {
  char* ptr = nullptr;
  uint64_t owner = 0;
};
std::mutex g_scratch_mu;
std::map<int, DeviceScratch>& scratch_table() {
  static std::map<int, DeviceScratch> t;
  return t;
}
int current_device() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  return dev;
}
}  // namespace

char* noalloc_scratch(size_t* bytes) {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  DeviceScratch& d = scratch_table()[dev];
  if (!d.ptr) {
    // once per device, with that device current: its own copy of the array
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) throw Failure(ST_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    d.ptr = static_cast<char*>(p);
    reg_add(p, ACR_NOALLOC_SCRATCH_BYTES);   // known to the host-side bounds check
  }
  if (bytes) *bytes = ACR_NOALLOC_SCRATCH_BYTES;
  return d.ptr;
}

uint64_t noalloc_owner() {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return scratch_table()[dev].owner;
}

void set_noalloc_owner(uint64_t id) {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  scratch_table()[dev].owner = id;
}

void Exec::check_range(const void* p, size_t bytes, const char* what) const {
  if (!checking || bytes == 0) return;
  std::lock_guard<std::mutex> lk(g_reg_mu);
  auto& r = registry();
  const uintptr_t a = (uintptr_t)p;
  auto it = r.upper_bound(a);
  if (p == nullptr || it == r.begin()) throw Failure(ST_HIP, std::string("bounds check: unknown pointer in ") + what);
  --it;
  if (a + bytes > it->first + it->second)
    throw Failure(ST_HIP, std::string("bounds check: access past allocation end in ") + what);
}

namespace {
inline size_t ext(int rows, int cols, int64_t ld) {
  if (rows <= 0 || cols <= 0) return 0;
  return (size_t)(cols - 1) * (size_t)ld + (size_t)rows;
}
}  // namespace

void Exec::init(hipStream_t s, const Allocator& a) {
  const char* ck = std::getenv("ACR_CHECK");
  checking = ck && ck[0] == '1';
  const char* tr = std::getenv("ACR_TRACE");
  trace = tr && tr[0] == '1';
  const char* gm = std::getenv("ACR_GRAM");
  gram_ok = !(gm && gm[0] == '0');
  fused_lds = kFusedLds;
  const char* sg = std::getenv("ACR_SVD_GLOBAL");
  svd_global = sg && sg[0] == '1';
  const char* pg = std::getenv("ACR_PCHOL_GLOBAL");
  pchol_global = pg && pg[0] == '1';
  const char* pl = std::getenv("ACR_PCHOL_LDS");
  pchol_lds = pl && pl[0] == '1';
  const char* iu = std::getenv("ACR_INVERSE_UNBLOCKED");
  inverse_unblocked = iu && iu[0] == '1';
  const char* gn = std::getenv("ACR_GEMM_NARROW");
  gemm_narrow = !(gn && gn[0] == '0');
  const char* lq = std::getenv("ACR_SVD_LQ");
  svd_lq = !(lq && lq[0] == '0');
  const char* pt = std::getenv("ACR_PCHOL_TILES");
  pchol_512 = pt && std::strcmp(pt, "512") == 0;
  pchol_mid = !(pt && std::strcmp(pt, "1024") == 0);
  const char* nm = std::getenv("ACR_NO_MERGE");
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    merge_cus = (nm && nm[0] == '1') ? 0 : cus;
  stream = s;
  al = a;
  ring_bytes_ = size_t(64) << 20;
  hip_check(hipHostMalloc((void**)&h_ring_, ring_bytes_, hipHostMallocDefault), "hipHostMalloc(ring)");
  d_ring_ = static_cast<char*>(dev_alloc(ring_bytes_));
  d_flags = static_cast<int*>(dev_alloc(NFLAGS * sizeof(int)));
  hip_check(hipHostMalloc((void**)&h_flags, NFLAGS * sizeof(int), hipHostMallocDefault), "hipHostMalloc(flags)");
  // side stream (default priority) for the long global-memory SVD stages
  if (hipStreamCreateWithFlags(&side_, hipStreamNonBlocking) != hipSuccess) side_ = nullptr;
  for (hipEvent_t& e : ev_) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
  d_svd_flops = static_cast<unsigned long long*>(dev_alloc(sizeof(unsigned long long)));
  hip_check(hipMemsetAsync(d_svd_flops, 0, sizeof(unsigned long long), stream), "hipMemsetAsync(svd flops)");
  clear_flags();
}

double Exec::device_svd_flops() {
  unsigned long long v = 0;
  if (!d_svd_flops) return 0.0;
  hip_check(hipMemcpyAsync(&v, d_svd_flops, sizeof(v), hipMemcpyDeviceToHost, stream), "hipMemcpyAsync(svd flops)");
  hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
  return (double)v;
}

void Exec::destroy() {
  (void)hipDeviceSynchronize();
  if (!pending_.empty()) resolve_timings();
  for (hipEvent_t e : event_pool_) (void)hipEventDestroy(e);
  event_pool_.clear();
  if (d_counters_) dev_free(d_counters_);
  d_counters_ = nullptr;
  for (void* p : oversized_) dev_free(p);
  oversized_.clear();
  if (h_ring_) (void)hipHostFree(h_ring_);
  if (h_flags) (void)hipHostFree(h_flags);
  if (d_ring_) dev_free(d_ring_);
  if (d_flags) dev_free(d_flags);
  if (d_svd_flops) dev_free(d_svd_flops);
  d_svd_flops = nullptr;
  if (side_) (void)hipStreamDestroy(side_);
  side_ = nullptr;
  for (hipEvent_t& e : ev_) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  h_ring_ = nullptr; h_flags = nullptr; d_ring_ = nullptr; d_flags = nullptr;
}

void* Exec::dev_alloc(size_t bytes) {
  void* p = nullptr;
  if (al.alloc) {
    p = al.alloc(bytes, al.ctx, stream);
    if (!p) throw Failure(ST_OOM, "allocator callback returned NULL");
  } else {
    const int dev = current_device();
    if (pool_enabled()) p = pool_take(dev, bytes);
    if (!p) {
      hipError_t e = hipMalloc(&p, bytes);
      if (e == hipErrorOutOfMemory && pool_enabled()) {
        (void)hipGetLastError();
        pool_release();
        e = hipMalloc(&p, bytes);
      }
      hip_check(e, "hipMalloc");
    }
  }
  reg_add(p, bytes);
  return p;
}

void Exec::dev_free(void* p) {
  if (!p) return;
  const size_t bytes = reg_del(p);
  if (al.release) {
    al.release(p, al.ctx, stream);
    return;
  }
  if (pool_enabled() && bytes > 0) {
    // the executor's streams are the only users of its buffers (solve streams
    // are synchronised before a handle's memory is released): once they are
    // idle the buffer can serve any later request
    (void)hipStreamSynchronize(stream);
    if (side_) (void)hipStreamSynchronize(side_);
    pool_put(current_device(), p, bytes);
    return;
  }
  (void)hipFree(p);  // hipFree waits for the device to finish with the memory
}

void Exec::sync() {
  hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
  if (side_) hip_check(hipStreamSynchronize(side_), "hipStreamSynchronize(side)");
  if (!pending_.empty()) resolve_timings();
}

const void* Exec::upload_bytes(const void* src, size_t bytes) {
  if (bytes == 0) return nullptr;
  if (rec_arena) {
    void* d = rec_arena->get(bytes);
    if (rec_image) {
      const size_t off = static_cast<const char*>(d) - rec_image_base;
      if (rec_image->size() < off + bytes) rec_image->resize(off + bytes);
      std::memcpy(rec_image->data() + off, src, bytes);
      return d;
    }
    hip_check(hipMemcpy(d, src, bytes, hipMemcpyHostToDevice), "hipMemcpy(plan tasks)");
    return d;
  }
  const size_t b = (bytes + 255) & ~size_t(255);
  if (b > ring_bytes_) {
    // oversized batch: a dedicated buffer released at the next sync point
    sync();
    void* d = dev_alloc(b);
    hip_check(hipMemcpy(d, src, bytes, hipMemcpyHostToDevice), "hipMemcpy(tasks)");
    oversized_.push_back(d);
    return d;
  }
  if (ring_off_ + b > ring_bytes_) {
    sync();  // every earlier launch that read the ring has completed
    ring_off_ = 0;
    for (void* p : oversized_) dev_free(p);
    oversized_.clear();
  }
  std::memcpy(h_ring_ + ring_off_, src, bytes);
  hip_check(hipMemcpyAsync(d_ring_ + ring_off_, h_ring_ + ring_off_, bytes, hipMemcpyHostToDevice, stream),
            "hipMemcpyAsync(tasks)");
  const void* d = d_ring_ + ring_off_;
  ring_off_ += b;
  return d;
}

void Exec::replay_timed(const std::vector<Recorded>& r, hipStream_t s) {
  hipStream_t saved = stream;
  stream = s;
  std::vector<Recorded>* saved_rec = rec;
  const long saved_launches = launches;
  rec = nullptr;
  for (const Recorded& x : r) {
    Work w = x.w;
    if (w.counter) w.counter = nullptr;   // device counters belong to the recording
    submit(x.f, w);
  }
  rec = saved_rec;
  stream = saved;
  launches = saved_launches;
}

void Exec::submit(std::function<void(hipStream_t)> f, const Work& w) {
  ++launches;
  if (rec) {
    rec->push_back(Recorded{f, w});
    return;
  }
  const bool timed = g_timing && w.cls;
  Pending p{};
  if (timed) {
    for (hipEvent_t* e : {&p.a, &p.b}) {
      if (!event_pool_.empty()) {
        *e = event_pool_.back();
        event_pool_.pop_back();
      } else {
        hip_check(hipEventCreate(e), "hipEventCreate");
      }
    }
    hip_check(hipEventRecord(p.a, stream), "hipEventRecord");
  }
  f(stream);
  hip_check(hipGetLastError(), "kernel launch");
  if (timed) {
    hip_check(hipEventRecord(p.b, stream), "hipEventRecord");
    p.w = w;
    pending_.push_back(p);
  }
}

void Exec::clear_flags() {
  hip_check(hipMemsetAsync(d_flags, 0, NFLAGS * sizeof(int), stream), "hipMemsetAsync(flags)");
}

void Exec::read_flags(int out[NFLAGS]) {
  hip_check(hipMemcpyAsync(h_flags, d_flags, NFLAGS * sizeof(int), hipMemcpyDeviceToHost, stream),
            "hipMemcpyAsync(flags)");
  sync();
  for (int i = 0; i < NFLAGS; ++i) out[i] = h_flags[i];
}

// Splits tasks by the local memory they need: one launch per size class of the
// LDS-resident kernel (so small problems are not limited by the occupancy of
// large ones), one launch of the global-memory kernel for the rest.  Classes
// whose tasks all fit on the chip at once at the occupancy of the largest one
// (cus compute units, `threads` per workgroup; 0: 256 up to kSmallLds, else
// 1024) share a launch: their workgroups would not have waited for each
// other, and a second launch of a few long tasks would serialise behind the
// first.
inline int wg_per_cu(size_t lds, int threads) {
  const int by_lds = lds > 0 ? (int)(kLdsPerCu / lds) : 64;
  const int by_threads = 2048 / threads;
  return std::max(1, std::min(by_lds, by_threads));
}

template <class Task, class Need, class Launch>
void bucketed(const std::vector<Task>& t, Need need, Launch launch, int cus = 0, int threads = 0) {
  static const size_t cls[] = {16 * 1024, 32 * 1024, 64 * 1024, 96 * 1024, kLdsBudget};
  std::vector<Task> b[6];
  size_t mx[5] = {0, 0, 0, 0, 0};
  for (const Task& x : t) {
    const size_t n = need(x);
    int c = 5;
    for (int i = 0; i < 5; ++i)
      if (n <= cls[i]) { c = i; break; }
    b[c].push_back(x);
    if (c < 5) mx[c] = std::max(mx[c], n);
  }
  for (int i = 4; i >= 0; --i) {
    if (b[i].empty()) continue;
    size_t lds = std::max<size_t>(mx[i], 16);
    std::vector<Task> group = std::move(b[i]);
    while (cus > 0) {
      int j = i - 1;
      while (j >= 0 && b[j].empty()) --j;
      if (j < 0) break;
      const int nt = threads ? threads : (lds <= kSmallLds ? 256 : 1024);
      if ((long)(group.size() + b[j].size()) > (long)cus * wg_per_cu(lds, nt)) break;
      group.insert(group.end(), b[j].begin(), b[j].end());
      b[j].clear();
      i = j;
    }
    launch(group, lds);
  }
  if (!b[5].empty()) launch(b[5], 0);
}

template <class T> void Exec::gemm(const std::vector<GemmTask>& t) {
  if (t.empty()) return;
  if (checking)
    for (auto& x : t) {
      if (x.m < 0 || x.n < 0 || x.k < 0) throw Failure(ST_HIP, "bounds check: negative gemm size");
      const size_t e = sizeof(T);
      check_range(x.A, e * (x.ta ? ext(x.k, x.m, x.lda) : ext(x.m, x.k, x.lda)), "gemm A");
      check_range(x.B, e * (x.tb ? ext(x.n, x.k, x.ldb) : ext(x.k, x.n, x.ldb)), "gemm B");
      check_range(x.C, e * ext(x.m, x.n, x.ldc), "gemm C");
      if ((x.ta ? x.lda < x.k : x.lda < x.m) && x.m * x.k > 0) throw Failure(ST_HIP, "bounds check: gemm lda");
      if ((x.tb ? x.ldb < x.n : x.ldb < x.k) && x.n * x.k > 0) throw Failure(ST_HIP, "bounds check: gemm ldb");
      if (x.ldc < x.m && x.m * x.n > 0) throw Failure(ST_HIP, "bounds check: gemm ldc");
    }
  // one launch per input kind: native-precision matrix cores, or 16-bit
  // inputs; FP32 outputs at most 32 columns wide in a launch of 128 x 32 tiles
  for (int mode = 0; mode < 4; ++mode) {
    std::vector<int> first, tile_task;
    std::vector<GemmTask> sel;
    int nt = 0;
    for (const GemmTask& x : t) {
      int m = (sizeof(T) != 4 || x.lowp < 0) ? 0 : (x.lowp > 0 ? x.lowp : prod_lowp);
      if (m == 0 && sizeof(T) == 4 && gemm_narrow && x.n <= 32) m = 3;
      if (m != mode) continue;
      first.push_back(nt);
      const int tiles = mode == 3 ? (x.m + 127) / 128 : ((x.m + 63) / 64) * ((x.n + 63) / 64);
      for (int j = 0; j < tiles; ++j) tile_task.push_back((int)sel.size());
      nt += tiles;
      sel.push_back(x);
      flops_gemm += 2.0 * x.m * x.n * (double)x.k;
    }
    if (nt == 0) continue;
    Work w;
    w.cls = (mode == 0 || mode == 3) ? "gemm" : (mode == 1 ? "gemm_bf16" : "gemm_f16");
    for (auto& x : sel) {
      w.flops += 2.0 * x.m * x.n * (double)x.k;
      w.bytes += sizeof(T) * ((double)x.m * x.k + (double)x.k * x.n + (double)x.m * x.n * (x.beta != 0.0 ? 2 : 1));
    }
    const GemmTask* dt;
    const int *dtt, *dft;
    upload3(sel, tile_task, first, &dt, &dtt, &dft);
    if (mode == 3)
      submit([=](hipStream_t s) { launch_gemm_narrow(dt, dtt, dft, nt, s); }, w);
    else
      submit([=](hipStream_t s) { launch_gemm_mfma<T>(dt, dtt, dft, nt, mode, s); }, w);
  }
}

template <class T> void Exec::seg_gemm(const std::vector<SegGemmTask>& t) {
  if (t.empty()) return;
  std::vector<int> first, tile_task;
  int nt = 0;
  Work w;
  w.cls = "seg_gemm";
  for (size_t i = 0; i < t.size(); ++i) {
    const SegGemmTask& x = t[i];
    if (x.nseg < 0 || x.nseg > kMaxSeg || x.m < 0 || x.n < 0) throw Failure(ST_HIP, "bounds check: seg gemm shape");
    const size_t e = sizeof(T);
    double ktot = 0;
    for (int q = 0; q < x.nseg; ++q) {
      if (x.k[q] < 0) throw Failure(ST_HIP, "bounds check: seg gemm k");
      const bool ta = (x.ta >> q) & 1;
      if (checking) {
        check_range(x.A[q], e * (ta ? ext(x.k[q], x.m, x.lda[q]) : ext(x.m, x.k[q], x.lda[q])), "seg gemm A");
        check_range(x.B[q], e * ext(x.k[q], x.n, x.ldb[q]), "seg gemm B");
      }
      if ((ta ? x.lda[q] < x.k[q] : x.lda[q] < x.m) && x.m * x.k[q] > 0) throw Failure(ST_HIP, "bounds check: seg lda");
      if (x.ldb[q] < x.k[q] && x.k[q] * x.n > 0) throw Failure(ST_HIP, "bounds check: seg ldb");
      ktot += x.k[q];
    }
    if (checking) check_range(x.C, e * ext(x.m, x.n, x.ldc), "seg gemm C");
    if (x.ldc < x.m && x.m * x.n > 0) throw Failure(ST_HIP, "bounds check: seg ldc");
    first.push_back(nt);
    const int tiles = ((x.m + 63) / 64) * ((x.n + 63) / 64);
    for (int j = 0; j < tiles; ++j) tile_task.push_back((int)i);
    nt += tiles;
    w.flops += 2.0 * x.m * x.n * ktot;
    w.bytes += e * ((double)x.m * ktot + ktot * x.n + (double)x.m * x.n * (x.beta != 0.0 ? 2 : 1));
  }
  flops_gemm += w.flops;
  if (nt == 0) return;
  const SegGemmTask* dt;
  const int *dtt, *dft;
  upload3(t, tile_task, first, &dt, &dtt, &dft);
  submit([=](hipStream_t s) { launch_seg_gemm<T>(dt, dtt, dft, nt, s); }, w);
}

template <class T> void Exec::copy(const std::vector<CopyTask>& t) {
  if (t.empty()) return;
  if (checking)
    for (auto& x : t) {
      const size_t e = sizeof(T);
      if (x.src) check_range(x.src, e * ext(x.m, x.n, x.lds), "copy src");
      check_range(x.dst, e * ext(x.m, x.n, x.ldd), "copy dst");
      if (x.rs) check_range(x.rs, e * x.m, "copy rs");
      if (x.cs) check_range(x.cs, e * x.n, "copy cs");
      if (x.ldd < x.m || (x.src && x.lds < x.m)) throw Failure(ST_HIP, "bounds check: copy ld");
    }
  Work w;
  w.cls = "copy";
  for (auto& x : t) w.bytes += sizeof(T) * (double)x.m * x.n * ((x.src ? 1 : 0) + 1 + (x.accumulate ? 1 : 0));
  // workgroups per task along y: enough that the launch has about 8192
  // workgroups (a single large copy spreads over the chip) and that no
  // workgroup takes more than 32 units of the largest task, at most that
  // task's units (short columns share a unit, so a launch of many small
  // blocks does not pay for idle workgroups)
  int64_t units = 1, total = 0;
  for (auto& x : t) {
    const int64_t u = copy_units(x.m, x.n);
    units = std::max<int64_t>(units, u);
    total += u;
  }
  const int n = (int)t.size();
  const int64_t per = (total + n - 1) / n;   // mean units per task
  const int64_t want = std::max<int64_t>({(8192 + n - 1) / n, (units + 31) / 32, std::min<int64_t>(per, 4)});
  const int gy = (int)std::min<int64_t>({units, want, 65535});
  const CopyTask* dt = upload(t);
  submit([=](hipStream_t s) { launch_copy<T>(dt, n, gy, s); }, w);
}

template <class T> void Exec::inverse(const std::vector<InvTask>& t) {
  if (t.empty()) return;
  if (checking)
    for (auto& x : t) {
      check_range(x.A, sizeof(T) * ext(x.s, x.s, x.lda), "inverse");
      if (x.lda < x.s) throw Failure(ST_HIP, "bounds check: inverse ld");
    }
  int mx = 0;
  for (auto& x : t) {
    mx = std::max(mx, x.s);
    flops_inv += 2.0 * x.s * x.s * (double)x.s;
  }
  Work w;
  w.cls = "inverse";
  for (auto& x : t) {
    w.flops += 2.0 * x.s * x.s * (double)x.s;
    w.bytes += 2.0 * sizeof(T) * x.s * (double)x.s;
  }
  const InvTask* dt = upload(t);
  const int n = (int)t.size();
  int* fl = d_flags;
  const bool ub = inverse_unblocked;
  submit([=](hipStream_t s) { launch_inverse<T>(dt, n, mx, fl, s, ub); }, w);
}

template <class T> void Exec::qr(const std::vector<QrTask>& t) {
  if (t.empty()) return;
  if (checking)
    for (auto& x : t) {
      check_range(x.A, sizeof(T) * ext(x.m, x.r, x.lda), "qr panel");
      check_range(x.tau, sizeof(T) * std::min(x.m, x.r), "qr tau");
      if (x.lda < x.m) throw Failure(ST_HIP, "bounds check: qr ld");
    }
  for (auto& x : t) {
    const double m = x.m, r = std::min(x.m, x.r);
    flops_qr += 2.0 * m * x.r * r - 2.0 / 3.0 * r * r * r;
  }
  bucketed(t, [](const QrTask& x) { return lds_bytes_qr(x, sizeof(T)); },
           [this](const std::vector<QrTask>& b, size_t lds) {
             Work w;
             w.cls = lds ? "qr_lds" : "qr";
             for (auto& x : b) {
               const double m = x.m, r = x.r, p = std::min(x.m, x.r);
               w.flops += 4.0 * m * r * p - 2.0 * p * p * (m + r) + 4.0 / 3.0 * p * p * p;
               w.bytes += 2.0 * sizeof(T) * m * r;
             }
             const QrTask* dt = upload(b);
             const int n = (int)b.size();
             submit([=](hipStream_t s) { launch_qr_lds<T>(dt, n, lds, s); }, w);
           },
           merge_cus);
}

template <class T> void Exec::svd(std::vector<SvdTask>& t, double eps, int* d_tvals) {
  if (t.empty()) return;
  if (checking)
    for (auto& x : t) {
      const size_t rw = x.mode == 1 ? sizeof(double) : sizeof(T);
      check_range(x.Ru, rw * ext(x.p, x.r, x.ldu), "svd Ru");
      check_range(x.Rv, rw * ext(x.q, x.r, x.ldv), "svd Rv");
      check_range(x.C, sizeof(double) * 2 * (size_t)x.p * x.q, "svd C");
      check_range(x.Y, sizeof(double) * 2 * (size_t)x.q * x.q, "svd Y");
      check_range(x.perm, sizeof(int) * x.q, "svd perm");
      check_range(x.sig, sizeof(double) * x.q, "svd sig");
      check_range(x.t_out, sizeof(int), "svd t");
      check_range(x.rank_out, sizeof(int), "svd rank");
      if (x.ldu < x.p || x.ldv < x.q) throw Failure(ST_HIP, "bounds check: svd ld");
      if (x.r < x.p || x.r < x.q) throw Failure(ST_HIP, "bounds check: svd core shape");
    }
  // the pivoted QR drops a trailing block of Frobenius norm at most delta
  // times the core's largest column norm (<= sigma_1): with delta = eps / 10
  // the compression error stays within 1.1 eps sigma_1, and only values within
  // eps sigma_1 / 10 of the threshold can change their side of it
  const double delta = eps > 0.0 ? 0.1 * eps : 0.0;
  int* fl = d_flags;
  for (auto& x : t) x.flop_ctr = d_svd_flops;
  std::vector<SvdTask> small, mid, big;
  std::vector<int> big_idx;
  for (size_t i = 0; i < t.size(); ++i) {
    // the blocked sweeps index a core with 32-bit offsets
    if (t[i].p >= 32768 || t[i].q >= 32768) throw Failure(ST_NOT_SUPPORTED, "compression core too large");
    if (svd_global) {
      big.push_back(t[i]);
      big_idx.push_back((int)i);
    } else if (svd_wave_ok(t[i])) {
      small.push_back(t[i]);
    } else if (lds_bytes_svd_block(t[i]) <= fused_lds) {
      mid.push_back(t[i]);
    } else {
      big.push_back(t[i]);
      big_idx.push_back((int)i);
    }
  }
  // left factors of a batch of finished cores
  auto left = [this](std::vector<SvdTask>& b) {
    if (b.empty()) return;
    int qr = 0, mn = 0;
    for (auto& x : b) {
      qr = std::max(qr, x.q + x.r);
      mn = std::max(mn, std::min(x.p, x.q));
    }
    int kc = 32;
    while (kc > 1 && (size_t)qr * kc * 8 > 64 * 1024) kc >>= 1;
    const int nchunks = (mn + kc - 1) / kc;
    const size_t lds = (size_t)qr * kc * 8;
    if (lds > kLdsBudget) throw Failure(ST_NOT_SUPPORTED, "core too large for the left-factor kernel");
    Work w;
    w.cls = "core_left";
    unsigned long long* ctr = g_timing ? counter_slot() : nullptr;
    w.counter = ctr;
    w.flops_per_count = 2.0;
    for (auto& x : b) w.bytes += (double)sizeof(T) * 0.5 * ((double)x.p + x.q) * x.r;
    const SvdTask* dt = upload(b);
    const int n = (int)b.size();
    submit([=](hipStream_t s) { launch_core_left<T>(dt, n, kc, nchunks, lds, ctr, s); }, w);
  };
  // one-workgroup cores: the kernels count the flops of their core product,
  // pivoted QR and sweeps
  auto fused = [this, delta, eps, fl](const std::vector<SvdTask>& b, size_t lds, bool wave) {
    Work w;
    w.cls = wave ? "svd_wave" : "svd_block";
    unsigned long long* ctr = g_timing ? counter_slot() : nullptr;
    std::vector<SvdTask> bb = b;
    for (auto& x : bb) {
      x.sweep_ctr = ctr;
      w.bytes += (double)sizeof(T) * 0.5 * ((double)x.p + x.q) * x.r;
    }
    w.counter = ctr;
    w.flops_per_count = 1.0;
    const SvdTask* dt = upload(bb);
    const int n = (int)bb.size();
    if (wave)
      submit([=](hipStream_t s) { launch_svd_wave<T>(dt, n, delta, eps, fl, lds, s); }, w);
    else
      submit([=](hipStream_t s) { launch_svd_block<T>(dt, n, delta, eps, fl, lds, s); }, w);
  };
  // Two-phase cores (pivoted QR, host read of the ranks t, Jacobi on W^T):
  // those whose C fits in LDS stay on the main stream; the global-memory ones
  // (few per launch, each one long) run on the side stream so that they overlap
  // the many small and mid-size cores instead of idling most of the chip.
  std::vector<SvdTask> two[2];
  std::vector<int> two_idx[2];
  for (size_t i = 0; i < big.size(); ++i) {
    const int g = (side_ && (svd_global || lds_bytes_qrcp(big[i]) > kLdsBudget)) ? 1 : 0;
    two[g].push_back(big[i]);
    two_idx[g].push_back(big_idx[i]);
  }
  for (auto& x : big) flops_svd += 2.0 * x.p * x.q * (double)x.r;
  auto qrcp_batch = [this, delta](const std::vector<SvdTask>& b, size_t lds) {
    Work w;
    w.cls = lds ? "qrcp_lds" : "qrcp";
    for (auto& x : b) {
      w.flops += 2.0 * x.p * x.q * (double)x.r;  // forming the core (pivoted QR added below)
      w.bytes += 8.0 * ((double)x.p + x.q) * x.r + 8.0 * x.q * std::min(x.p, x.q);
    }
    const SvdTask* dt = upload(b);
    const int n = (int)b.size();
    int max_q = 1;
    for (auto& x : b) max_q = std::max(max_q, x.q);
    submit([=](hipStream_t s) { launch_qrcp<T>(dt, n, delta, lds, max_q, s); }, w);
  };
  auto jacobi_batch = [this, eps, fl](const std::vector<SvdTask>& b, size_t lds) {
    Work w;
    w.cls = lds ? "jacobi_lds" : "jacobi";
    unsigned long long* ctr = g_timing ? counter_slot() : nullptr;
    std::vector<SvdTask> bb = b;
    // the kernels add the flops their sweeps did (inner products of every
    // visit, rotations where applied) to the counter; algorithmic bytes: W^T
    // (q x t) read once, at most t right vectors of length q written
    for (auto& x : bb) {
      x.sweep_ctr = ctr;
      w.bytes += 2.0 * 8.0 * (double)x.q * (double)x.tc;
    }
    w.counter = ctr;
    w.flops_per_count = 1.0;
    if (trace) {
      // vectors (rows q) and columns (rank t) of the launch, by quartile
      std::vector<int> qs, ts;
      for (auto& x : bb) {
        qs.push_back(x.q);
        ts.push_back(x.tc);
      }
      std::sort(qs.begin(), qs.end());
      std::sort(ts.begin(), ts.end());
      const size_t m = qs.size();
      std::fprintf(stderr, "[acr] jacobi lds=%zu cores=%zu q %d/%d/%d/%d t %d/%d/%d/%d\n", lds, m, qs[0],
                   qs[m / 4], qs[m / 2], qs[m - 1], ts[0], ts[m / 4], ts[m / 2], ts[m - 1]);
    }
    // threads for one pass per round over every core's column pairs: 8 lanes
    // per pair for vectors up to 128 long, 16 for longer ones (the blocked
    // sweeps in global memory: 1024 threads once a vector exceeds the
    // register-resident visit)
    int threads = 0;
    for (auto& x : bb) {
      const int need = lds == 0 ? (x.q > kJBRegRows ? 1024 : 512) : (x.q <= 128 ? 8 : 16) * ((x.tc + 1) / 2);
      threads = std::max(threads, need);
    }
    const SvdTask* dt = upload(bb);
    const int n = (int)bb.size();
    submit([=](hipStream_t s) { launch_jacobi<T>(dt, n, eps, fl, lds, threads, s); }, w);
  };
  // numerical ranks found by the pivoted QR, read back per stream
  std::vector<int> tv[2];
  auto read_ranks = [&](int g) {
    tv[g].resize(t.size());
    hip_check(hipMemcpyAsync(tv[g].data(), d_tvals, t.size() * sizeof(int), hipMemcpyDeviceToHost, stream),
              "hipMemcpyAsync(core ranks)");
    hip_check(hipEventRecord(ev_[g], stream), "hipEventRecord");
  };
  auto rank_stage = [&](int g) {
    hip_check(hipEventSynchronize(ev_[g]), "hipEventSynchronize(core ranks)");
    double qf = 0;
    for (size_t i = 0; i < two[g].size(); ++i) {
      const int k = tv[g][two_idx[g][i]];
      two[g][i].tc = k;
      const double p = two[g][i].p, q = two[g][i].q;
      qf += 4.0 * p * q * k - 2.0 * (double)k * k * (p + q) + 4.0 / 3.0 * (double)k * k * k;
    }
    flops_svd += qf;
    // the pivoted QR stopped at rank t: add its Householder work to the timing record
    for (auto it = pending_.rbegin(); it != pending_.rend(); ++it)
      if (it->w.cls && std::strncmp(it->w.cls, "qrcp", 4) == 0) { it->w.flops += qf; break; }
  };
  const bool split = !two[1].empty();
  if (split) {
    // side stream: starts after everything submitted so far (the stack QRs)
    hip_check(hipEventRecord(ev_[2], stream), "hipEventRecord");
    hip_check(hipStreamWaitEvent(side_, ev_[2], 0), "hipStreamWaitEvent");
    std::swap(stream, side_);
    qrcp_batch(two[1], 0);
    read_ranks(1);
    std::swap(stream, side_);
  }
  // main stream: pivoted QR of the LDS cores first (their ranks come back
  // early), then the one-workgroup cores
  bucketed(two[0], [](const SvdTask& x) { return lds_bytes_qrcp(x); }, qrcp_batch, merge_cus);
  if (!two[0].empty()) read_ranks(0);
  bucketed(small, [](const SvdTask& x) { return lds_bytes_svd_wave(x, sizeof(T)); },
           [&](const std::vector<SvdTask>& b, size_t lds) { fused(b, lds, true); }, merge_cus, 64);
  bucketed(mid, [](const SvdTask& x) { return lds_bytes_svd_block(x); },
           [&](const std::vector<SvdTask>& b, size_t lds) { fused(b, lds, false); }, merge_cus);
  small.insert(small.end(), mid.begin(), mid.end());
  left(small);
  if (!two[0].empty()) {
    rank_stage(0);
    bucketed(two[0], [](const SvdTask& x) { return lds_bytes_jacobi(x); }, jacobi_batch, merge_cus);
    left(two[0]);
  }
  if (split) {
    rank_stage(1);
    std::swap(stream, side_);
    // Cores whose W^T (q x t) exceeds LDS but whose t x t triangle fits, with
    // q > t: W^T = Q2 R2 (Householder QR in place), the scalar LDS sweeps on
    // the columns of R2 (R2 J = Zr Sigma with the rotations J and values of
    // W^T's sweeps), then Z = Q2 [Zr; 0].  The workspace C of the core (free
    // once the pivoted QR has written W^T) holds R2, Zr and the reflector
    // scales: 2 t^2 + t <= 2 p q doubles as p >= t and q > t.  (Blocked
    // sweeps on R2 for triangles beyond LDS measured slower than on W^T: the
    // QR and the reflector application lengthen the side stream.)
    std::vector<SvdTask> glob, red, redj;
    std::vector<QrTask> rq;
    std::vector<TriCopyTask> rc;
    std::vector<ApplyQTask> ra;
    for (auto& x : two[1]) {
      const int tt = x.tc;
      if (svd_lq && tt > 0 && x.q > tt && (size_t)tt * tt * 8 <= kLdsBudget) {
        double* buf = x.C;
        double* tau = x.C + 2 * (size_t)tt * tt;
        rq.push_back(QrTask{x.Y, tau, x.q, x.q, tt});
        rc.push_back(TriCopyTask{x.Y, buf, x.q, tt});
        SvdTask r = x;
        r.q = tt;
        r.Y = buf;
        redj.push_back(r);
        ApplyQTask aq;
        aq.Aq = x.Y; aq.tau = tau; aq.Z = buf + (size_t)tt * tt; aq.out = x.Y + (size_t)x.q * x.q;
        aq.lda = x.q; aq.ldz = tt; aq.ldo = x.q; aq.m = x.q; aq.p = tt; aq.k = tt;
        ra.push_back(aq);
        red.push_back(x);
      } else {
        glob.push_back(x);
      }
    }
    if (!redj.empty()) {
      qr<double>(rq);
      tri_copy(rc);
      bucketed(redj, [](const SvdTask& x) { return lds_bytes_jacobi(x); }, jacobi_batch, merge_cus);
      applyq<double>(ra);
    }
    if (svd_global) jacobi_batch(glob, 0);
    else bucketed(glob, [](const SvdTask& x) { return lds_bytes_jacobi(x); }, jacobi_batch, merge_cus);
    left(two[1]);
    hip_check(hipEventRecord(ev_[2], stream), "hipEventRecord");
    std::swap(stream, side_);
    hip_check(hipStreamWaitEvent(stream, ev_[2], 0), "hipStreamWaitEvent");
  }
  if (trace) {
    // sweep work of the two-kernel cores (rows q times t^2 columns pairs),
    // split by the ratio q / t of their rows to their pivoted-QR rank
    int mq = 0, mt = 0;
    double wk[4] = {0, 0, 0, 0};
    for (int g = 0; g < 2; ++g)
      for (auto& x : two[g]) {
        mq = std::max(mq, x.q);
        mt = std::max(mt, x.tc);
        const double ratio = x.tc > 0 ? (double)x.q / x.tc : 0.0;
        wk[ratio < 1.5 ? 0 : ratio < 2.0 ? 1 : ratio < 3.0 ? 2 : 3] += (double)x.q * x.tc * x.tc;
      }
    std::fprintf(stderr,
                 "[acr] svd %s fused=%zu two-kernel lds=%zu global=%zu max_q=%d max_t=%d "
                 "sweep work q/t<1.5:%.3g 1.5-2:%.3g 2-3:%.3g >3:%.3g\n",
                 trace_tag, small.size(), two[0].size(), two[1].size(), mq, mt, wk[0], wk[1], wk[2], wk[3]);
  }
}

template <class T> void Exec::applyq(const std::vector<ApplyQTask>& t) {
  if (t.empty()) return;
  if (checking)
    for (auto& x : t) {
      check_range(x.Aq, sizeof(T) * ext(x.m, x.p, x.lda), "applyq reflectors");
      check_range(x.tau, sizeof(T) * x.p, "applyq tau");
      check_range(x.Z, sizeof(double) * ext(x.p, x.k, x.ldz), "applyq Z");
      check_range(x.out, sizeof(T) * ext(x.m, x.k, x.ldo), "applyq out");
      if (x.p > x.m || x.ldo < x.m || x.lda < x.m) throw Failure(ST_HIP, "bounds check: applyq shape");
    }
  for (auto& x : t) flops_qr += 4.0 * x.m * x.p * (double)x.k;
  bucketed(t, [](const ApplyQTask& x) { return lds_bytes_applyq(x, sizeof(T)); },
           [this](const std::vector<ApplyQTask>& b, size_t lds) {
             Work w;
             w.cls = lds ? "applyq_lds" : "applyq";
             for (auto& x : b) {
               w.flops += 4.0 * x.m * x.p * (double)x.k;
               w.bytes += sizeof(T) * ((double)x.m * x.p + (double)x.m * x.k) + 8.0 * x.p * x.k;
             }
             const ApplyQTask* dt = upload(b);
             const int n = (int)b.size();
             submit([=](hipStream_t s) { launch_applyq_lds<T>(dt, n, lds, s); }, w);
           },
           merge_cus);
}

template <class T> void Exec::gram(const std::vector<GramTask>& t) {
  if (t.empty()) return;
  std::vector<int> first(t.size()), tile_task;
  int nt = 0;
  for (size_t i = 0; i < t.size(); ++i) {
    const GramTask& x = t[i];
    // the reduction indexes the r x r partials with 32-bit integers
    if ((int64_t)x.r * x.r > 0x7fffffff) throw Failure(ST_NOT_SUPPORTED, "stack too wide for the Gram kernels");
    if (checking) {
      check_range(x.A, sizeof(T) * ext(x.m, x.r, x.lda), "gram A");
      const int nch = (x.m + x.rows_per_chunk - 1) / x.rows_per_chunk;
      check_range(x.part, sizeof(double) * (size_t)nch * x.r * x.r, "gram part");
      check_range(x.G, sizeof(double) * (size_t)x.r * x.r, "gram G");
    }
    first[i] = nt;
    // one wavefront per (row chunk, pair of 32-column blocks), four per workgroup
    const int nb = (x.r + 31) / 32, nch = (x.m + x.rows_per_chunk - 1) / x.rows_per_chunk;
    const int tiles = (nch * nb * (nb + 1) / 2 + 3) / 4;
    for (int j = 0; j < tiles; ++j) tile_task.push_back((int)i);
    nt += tiles;
    flops_qr += (double)x.m * x.r * x.r;
  }
  Work w;
  w.cls = "gram";
  for (auto& x : t) {
    w.flops += (double)x.m * x.r * (x.r + 1);
    w.bytes += sizeof(T) * (double)x.m * x.r + 8.0 * x.r * x.r * ((x.m + x.rows_per_chunk - 1) / x.rows_per_chunk);
  }
  const GramTask* dt;
  const int *dtt, *dft;
  upload3(t, tile_task, first, &dt, &dtt, &dft);
  const int n = (int)t.size();
  // reduction: about 4096 workgroups per launch, at most 16 upper-triangle
  // tiles of the widest stack per workgroup
  int max_tiles = 1;
  for (auto& x : t) {
    const int nb = (x.r + 31) / 32;
    max_tiles = std::max(max_tiles, nb * (nb + 1) / 2);
  }
  const int rw = std::min({max_tiles, std::max((4096 + n - 1) / n, (max_tiles + 15) / 16), 65535});
  submit([=](hipStream_t s) { launch_gram<T>(dt, n, dtt, dft, nt, rw, s); }, w);
}

void Exec::pchol(const std::vector<PcholTask>& t, double tol) {
  if (t.empty()) return;
  for (auto& x : t) {
    check_range(x.G, sizeof(double) * (size_t)x.r * x.r, "pchol G");
    check_range(x.L, sizeof(double) * (size_t)x.r * x.r, "pchol L");
    check_range(x.perm, sizeof(int) * x.r, "pchol perm");
    check_range(x.d, sizeof(double) * x.r, "pchol d");
    check_range(x.rank_out, sizeof(int), "pchol rank");
    flops_qr += (double)x.r * x.r * x.r / 3.0;
  }
  // Gram matrices of order up to kPcholReg take the register-tiled kernel
  // (ACR_PCHOL_LDS=1: those whose packed lower triangle fits in LDS take the
  // right-looking LDS kernel instead), wider ones the left-looking one with L
  // in global memory; two launches at most per kind (finer size buckets
  // serialise the batch).  Orders up to kPcholRegMid take 5 x 5 tiles on 512
  // threads (their at most 465 tiles would leave over half of a 1024-thread
  // workgroup idle in every step), orders up to kPcholReg1024 5 x 5 tiles on
  // 1024 threads (at n = 128 the class took 287 ms per factorisation against
  // 333 ms with 8 x 8 tiles on 512 threads), orders up to kPcholReg 8 x 8
  // tiles (they went to the left-looking kernel before).  ACR_PCHOL_TILES=512
  // takes 8 x 8 tiles for every order above kPcholRegSmall, =1024 keeps the
  // orders up to kPcholRegMid on 1024 threads.
  std::vector<PcholTask> packed, wide, reg_small, reg_mid, reg_large, reg_big;
  int max_r = 1;
  for (auto& x : t) {
    if (!pchol_global && pchol_lds && lds_bytes_pchol_packed(x.r) <= kLdsBudget) {
      packed.push_back(x);
    } else if (!pchol_global && x.r <= kPcholReg) {
      (x.r <= kPcholRegSmall                   ? reg_small
       : pchol_512                             ? reg_big
       : x.r <= kPcholRegMid && pchol_mid      ? reg_mid
       : x.r <= kPcholReg1024                  ? reg_large
                                               : reg_big)
          .push_back(x);
    } else {
      wide.push_back(x);
      max_r = std::max(max_r, x.r);
    }
  }
  // the small kind joins the 1024-thread launch when that holds them all at
  // once (a second launch of a few long tasks would wait for the first)
  if (merge_cus > 0 && !reg_small.empty() && !reg_large.empty() &&
      (long)(reg_small.size() + reg_large.size()) <=
          (long)merge_cus * wg_per_cu(lds_bytes_pchol_reg(kPcholReg1024), 1024)) {
    reg_large.insert(reg_large.end(), reg_small.begin(), reg_small.end());
    reg_small.clear();
  }
  for (auto* b : {&reg_small, &reg_mid, &reg_large, &reg_big}) {
    if (b->empty()) continue;
    Work w;
    w.cls = "pchol";
    for (auto& x : *b) {
      w.flops += (double)x.r * x.r * x.r / 3.0;
      w.bytes += 16.0 * x.r * x.r;
    }
    const PcholTask* dt = upload(*b);
    const int n = (int)b->size();
    const int kind = b == &reg_small ? 0 : b == &reg_mid ? 3 : b == &reg_large ? 2 : 1;
    int rmax = 1;
    for (auto& x : *b) rmax = std::max(rmax, x.r);
    submit([=](hipStream_t s) { launch_pchol_reg(dt, n, rmax, tol, kind, s); }, w);
  }
  if ((size_t)max_r * (sizeof(double) + sizeof(int)) > kLdsBudget)
    throw Failure(ST_NOT_SUPPORTED, "stack too wide for the pivoted Cholesky kernel");
  auto launch = [&](const std::vector<PcholTask>& b, size_t lds) {
    Work w;
    w.cls = "pchol";
    for (auto& x : b) {
      w.flops += (double)x.r * x.r * x.r / 3.0;
      w.bytes += 16.0 * x.r * x.r;
    }
    const PcholTask* dt = upload(b);
    const int n = (int)b.size();
    submit([=](hipStream_t s) { launch_pchol(dt, n, max_r, tol, lds, s); }, w);
  };
  // small Gram matrices (packed triangle within kSmallLds) in a launch of
  // 256-thread workgroups of their own, the others in 1024-thread ones
  std::vector<PcholTask> small, large;
  size_t lds_small = 0, lds_large = 0;
  for (auto& x : packed) {
    const size_t b = lds_bytes_pchol_packed(x.r);
    if (b <= kSmallLds) {
      small.push_back(x);
      lds_small = std::max(lds_small, b);
    } else {
      large.push_back(x);
      lds_large = std::max(lds_large, b);
    }
  }
  if (!small.empty()) launch(small, lds_small);
  if (!large.empty()) launch(large, lds_large);
  if (!wide.empty()) launch(wide, 0);
}

void Exec::tri_copy(const std::vector<TriCopyTask>& t) {
  if (t.empty()) return;
  for (auto& x : t) {
    check_range(x.src, sizeof(double) * ext(x.n, x.n, x.lds), "tri_copy source");
    check_range(x.dst, sizeof(double) * 2 * (size_t)x.n * x.n, "tri_copy destination");
  }
  const TriCopyTask* dt = upload(t);
  const int n = (int)t.size();
  submit([=](hipStream_t s) { launch_tri_copy(dt, n, s); });
}

void Exec::materialize_r(const std::vector<PcholTask>& t) {
  if (t.empty()) return;
  for (auto& x : t) check_range(x.R, sizeof(double) * (size_t)x.r1 * x.r, "materialize R");
  // about 4096 workgroups per launch, at most 16 32 x 32 tiles of the largest
  // R per workgroup
  int max_tiles = 1;
  for (auto& x : t) max_tiles = std::max(max_tiles, ((x.r1 + 31) / 32) * ((x.r + 31) / 32));
  const int n = (int)t.size();
  const int wgs = std::min({max_tiles, std::max((4096 + n - 1) / n, (max_tiles + 15) / 16), 65535});
  const PcholTask* dt = upload(t);
  submit([=](hipStream_t s) { launch_materialize_r(dt, n, wgs, s); });
}

template <class T> void Exec::wtilde(const std::vector<WtTask>& t) {
  if (t.empty()) return;
  for (auto& x : t) {
    check_range(x.W, sizeof(T) * (size_t)x.r * x.k, "wtilde W");
    check_range(x.Z, sizeof(double) * ext(x.r1, x.k, x.ldz), "wtilde Z");
    check_range(x.L, sizeof(double) * (size_t)x.r * x.r, "wtilde L");
    check_range(x.perm, sizeof(int) * x.r, "wtilde perm");
  }
  Work w;
  w.cls = "wtilde";
  for (auto& x : t) {
    w.flops += (double)x.r1 * x.r1 * x.k;
    w.bytes += 8.0 * x.r1 * x.r1 / 2 + sizeof(T) * (double)x.r * x.k;
  }
  int r1max = 1, kmax = 0;
  for (auto& x : t) {
    if (x.r1 > x.r || x.r1 < 0) throw Failure(ST_HIP, "bounds check: wtilde rank");
    r1max = std::max(r1max, x.r1);
    kmax = std::max(kmax, x.k);
  }
  // chunk of right-hand sides and the 32 x 32 diagonal block of L in LDS, at
  // most 64 KiB so that two workgroups share a compute unit
  int kc = 64;
  while (kc > 1 && (size_t)r1max * kc * 8 + 32 * 32 * 8 > 64 * 1024) kc >>= 1;
  const size_t lds = (size_t)r1max * kc * 8 + 32 * 32 * 8;
  if (lds > kLdsBudget) throw Failure(ST_NOT_SUPPORTED, "rank too large for the back-substitution kernel");
  const int nchunks = (kmax + kc - 1) / kc;
  const WtTask* dt = upload(t);
  const int n = (int)t.size();
  submit([=](hipStream_t s) { launch_wtilde<T>(dt, n, kc, nchunks, lds, s); }, w);
}

template <class T> void Exec::inner(const std::vector<InnerTask>& t) {
  if (t.empty()) return;
  std::vector<int> first(t.size()), wave_task;
  int nw = 0;
  for (size_t i = 0; i < t.size(); ++i) {
    const InnerTask& x = t[i];
    if (checking) {
      check_range(x.V, sizeof(T) * ext(x.rows, x.k, x.ldv), "inner V");
      check_range(x.x, sizeof(T) * ext(x.rows, x.c, x.ldx), "inner x");
      check_range(x.t, sizeof(T) * (size_t)x.k * x.c, "inner t");
    }
    first[i] = nw;
    for (int j = 0; j < x.k; ++j) wave_task.push_back((int)i);
    nw += x.k;
  }
  Work w;
  w.cls = "solve_inner";
  for (auto& x : t) {
    w.flops += 2.0 * x.rows * x.k * (double)x.c;
    w.bytes += sizeof(T) * ((double)x.rows * x.k + (double)x.rows * x.c + (double)x.k * x.c);
  }
  constexpr int VW = 16 / sizeof(T);
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  bool vec = true;
  for (auto& x : t)
    vec = vec && x.rows % VW == 0 && x.ldv % VW == 0 && x.ldx % VW == 0 && al(x.V) && al(x.x);
  const InnerTask* dt;
  const int *dwt, *dfw;
  upload3(t, wave_task, first, &dt, &dwt, &dfw);
  submit([=](hipStream_t s) { launch_inner<T>(dt, dwt, dfw, nw, vec, s); }, w);
}

template <class T> void Exec::apply_leaf(const std::vector<LeafTask>& t) {
  if (t.empty()) return;
  if (checking)
    for (auto& x : t) {
      check_range(x.y, sizeof(T) * ext(x.n, x.c, x.ldy), "leaf y");
      if (x.yin) check_range(x.yin, sizeof(T) * ext(x.n, x.c, x.ldy), "leaf yin");
      for (int q = 0; q < x.nterm; ++q) {
        const LeafTerm& m = x.term[q];
        check_range(m.x, sizeof(T) * ext(x.n, x.c, m.ldx), "leaf x");
        if (m.diag) check_range(m.diag, sizeof(T) * x.n, "leaf diag");
        else check_range(m.leaf, sizeof(T) * (size_t)x.n * x.n, "leaf matrix");
        for (int d = 0; d < m.nd; ++d) {
          check_range(m.up[d], sizeof(T) * ext(x.n, m.kd[d], m.ldu[d]), "leaf U slice");
          check_range(m.tp[d], sizeof(T) * (size_t)m.kd[d] * x.c, "leaf t");
        }
      }
    }
  Work w;
  w.cls = "solve_leaf";
  for (auto& x : t) {
    double el = (double)x.n * x.c * ((x.yin && x.beta != 0.0) ? 2 : 1);
    for (int q = 0; q < x.nterm; ++q) {
      const LeafTerm& m = x.term[q];
      double mat = m.diag ? x.n : (double)x.n * x.n;
      for (int d = 0; d < m.nd; ++d) mat += (double)x.n * m.kd[d];
      w.flops += 2.0 * mat * x.c;
      el += mat + (double)x.n * x.c;
    }
    w.bytes += sizeof(T) * el;
  }
  constexpr int VW = 16 / sizeof(T);
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  bool vec = true;
  for (auto& x : t) {
    vec = vec && x.n > 0 && x.n % VW == 0 && x.n / VW <= 256 && x.ldy % VW == 0 && al(x.y) && (!x.yin || al(x.yin));
    for (int q = 0; q < x.nterm && vec; ++q) {
      const LeafTerm& m = x.term[q];
      vec = !m.trans && m.ldx % VW == 0 && al(m.x) && (m.diag ? al(m.diag) : al(m.leaf));
      for (int d = 0; d < m.nd && vec; ++d) vec = m.ldu[d] % VW == 0 && al(m.up[d]);
    }
  }
  const LeafTask* dt = upload(t);
  const int n = (int)t.size();
  submit([=](hipStream_t s) { launch_apply_leaf<T>(dt, n, vec, s); }, w);
}

#define ACR_EXEC_INST(T)                                              \
  template void Exec::gemm<T>(const std::vector<GemmTask>&);          \
  template void Exec::copy<T>(const std::vector<CopyTask>&);          \
  template void Exec::seg_gemm<T>(const std::vector<SegGemmTask>&);   \
  template void Exec::inverse<T>(const std::vector<InvTask>&);        \
  template void Exec::qr<T>(const std::vector<QrTask>&);              \
  template void Exec::svd<T>(std::vector<SvdTask>&, double, int*);   \
  template void Exec::applyq<T>(const std::vector<ApplyQTask>&);     \
  template void Exec::gram<T>(const std::vector<GramTask>&);         \
  template void Exec::wtilde<T>(const std::vector<WtTask>&);         \
  template void Exec::inner<T>(const std::vector<InnerTask>&);       \
  template void Exec::apply_leaf<T>(const std::vector<LeafTask>&);
ACR_EXEC_INST(float)
ACR_EXEC_INST(double)

}  // namespace acr
