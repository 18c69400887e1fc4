// Host-side structures of the library: cluster tree, device arenas, the
// launch executor and the weak-admissibility (HODLR) matrix handles.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "acr.h"
#include "kern.h"
#include "plan.h"

namespace acr {

// Internal failure carried to the C boundary as a status code.
struct Failure : std::runtime_error {
  int status;
  Failure(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

enum : int {
  ST_SUCCESS = 0, ST_INVALID = 1, ST_OOM = 2, ST_HIP = 3, ST_SINGULAR = 4,
  ST_RANK = 5, ST_NOT_CONVERGED = 6, ST_NOT_SUPPORTED = 7,
};

void hip_check(hipError_t e, const char* what);

// The fixed device scratch of the no-allocation solve on the current device
// (acquired once per device; *bytes = its size).  Throws on failure.
char* noalloc_scratch(size_t* bytes);
// Identifier of the no-allocation plan whose task arrays the current device's
// scratch holds (0 = none); set after a plan uploads them.
uint64_t noalloc_owner();
void set_noalloc_owner(uint64_t id);

struct Allocator {
  void* (*alloc)(size_t bytes, void* ctx, hipStream_t s) = nullptr;
  void (*release)(void* p, void* ctx, hipStream_t s) = nullptr;
  void* ctx = nullptr;
};

class Exec;

// Chunked bump allocator of device memory with stack-like marks.
class Arena {
 public:
  Arena() = default;
  void init(Exec* ex, size_t chunk) { ex_ = ex; chunk_ = chunk; }
  // Bump allocation inside one caller-owned device region of `bytes`: never
  // allocates; a request past its end throws (status invalid value).
  void init_fixed(void* base, size_t bytes);
  void* get(size_t bytes);
  template <class T> T* get_n(size_t n) { return static_cast<T*>(get(n * sizeof(T))); }
  struct Mark { size_t ci, off; };
  Mark mark() const { return {ci_, off_}; }
  void release(Mark m) { ci_ = m.ci; off_ = m.off; }
  void reset() { ci_ = 0; off_ = 0; }
  void free_all();
  size_t used() const;
  size_t reserved() const;
 private:
  Exec* ex_ = nullptr;
  size_t chunk_ = 0;
  std::vector<std::pair<char*, size_t>> chunks_;
  size_t ci_ = 0, off_ = 0;
  bool fixed_ = false;
};

// Algorithmic work of one launch, for the per-kernel timing table: flops and
// bytes counted from the task shapes (what the method must move or compute),
// optionally completed from a device counter the kernel fills in.
struct Work {
  const char* cls = nullptr;
  double flops = 0, bytes = 0;
  unsigned long long* counter = nullptr;
  double flops_per_count = 0, bytes_per_count = 0;
};

// Frees the device buffers kept for reuse (default allocator); returns bytes.
size_t release_cached_memory();

// Process-wide switch and table of per-kernel-class event timings.
void timing_enable(int level);   // 0 off, 1 factorisation launches, 2 also solve replays
bool timing_enabled();
bool solve_timing_enabled();
int timing_report(acr_kernel_time_t* out, int cap);

// Launch executor: uploads task arrays and launches, or records the launches
// of a solve into a replayable list (captured into a HIP graph by the caller).
class Exec {
 public:
  hipStream_t stream = nullptr;
  Allocator al;
  int* d_flags = nullptr;
  int* h_flags = nullptr;
  unsigned long long* d_svd_flops = nullptr;   // SVD flops counted by the kernels
  struct Recorded {
    std::function<void(hipStream_t)> f;
    Work w;
  };
  std::vector<Recorded>* rec = nullptr;
  Arena* rec_arena = nullptr;
  // With rec_arena set: when rec_image is set too, task arrays are not copied
  // to the device while recording; their bytes go to *rec_image at their
  // offset from rec_image_base, for the caller to upload stream-ordered.
  std::vector<char>* rec_image = nullptr;
  const char* rec_image_base = nullptr;

  void init(hipStream_t s, const Allocator& a);
  void destroy();
  void* dev_alloc(size_t bytes);
  void dev_free(void* p);
  void sync();
  // Device copy of a host array: the staging ring (immediate mode) or the
  // recording arena (recorded solves keep their task arrays for replay).
  const void* upload_bytes(const void* src, size_t bytes);
  template <class Task> const Task* upload(const std::vector<Task>& v) {
    return static_cast<const Task*>(upload_bytes(v.data(), v.size() * sizeof(Task)));
  }
  // One upload of a launch's task array and its two index arrays (one copy
  // dispatch instead of three); each array starts on a 16-byte boundary.
  template <class Task>
  void upload3(const std::vector<Task>& a, const std::vector<int>& b, const std::vector<int>& c, const Task** da,
               const int** db, const int** dc) {
    const size_t ob = (a.size() * sizeof(Task) + 15) & ~size_t(15);
    const size_t oc = ob + ((b.size() * sizeof(int) + 15) & ~size_t(15));
    std::vector<char> buf(oc + c.size() * sizeof(int));
    std::memcpy(buf.data(), a.data(), a.size() * sizeof(Task));
    std::memcpy(buf.data() + ob, b.data(), b.size() * sizeof(int));
    std::memcpy(buf.data() + oc, c.data(), c.size() * sizeof(int));
    const char* d = static_cast<const char*>(upload_bytes(buf.data(), buf.size()));
    *da = reinterpret_cast<const Task*>(d);
    *db = reinterpret_cast<const int*>(d + ob);
    *dc = reinterpret_cast<const int*>(d + oc);
  }
  void submit(std::function<void(hipStream_t)> f, const Work& w = Work{});
  // Eager replay of recorded launches on `s`, each timed like a submitted one
  // (used instead of the graph while the per-kernel timing table is on).
  void replay_timed(const std::vector<Recorded>& r, hipStream_t s);
  unsigned long long* counter_slot();   // zeroed device counter for one launch
  void resolve_timings();               // after the stream is idle
  void read_flags(int out[NFLAGS]);
  double device_svd_flops();            // synchronizes the stream
  void clear_flags();

  template <class T> void gemm(const std::vector<GemmTask>& t);
  template <class T> void seg_gemm(const std::vector<SegGemmTask>& t);
  template <class T> void copy(const std::vector<CopyTask>& t);
  template <class T> void inverse(const std::vector<InvTask>& t);
  template <class T> void qr(const std::vector<QrTask>& t);
  // d_tvals: device array of the tasks' t_out values (contiguous, in task order)
  template <class T> void svd(std::vector<SvdTask>& t, double eps, int* d_tvals);
  template <class T> void applyq(const std::vector<ApplyQTask>& t);
  void tri_copy(const std::vector<TriCopyTask>& t);
  template <class T> void gram(const std::vector<GramTask>& t);
  void pchol(const std::vector<PcholTask>& t, double tol);
  void materialize_r(const std::vector<PcholTask>& t);
  template <class T> void wtilde(const std::vector<WtTask>& t);
  template <class T> void inner(const std::vector<InnerTask>& t);
  template <class T> void apply_leaf(const std::vector<LeafTask>& t);

  // Host-side bounds check of every task against the live device allocations
  // (enabled with ACR_CHECK=1): a task that would touch memory outside one
  // allocation raises before anything is launched.
  bool checking = false;
  bool trace = false;          // ACR_TRACE=1: one line per compression batch on stderr
  bool gram_ok = true;         // ACR_GRAM=0 forces Householder compression everywhere
  size_t fused_lds = 0;        // one-workgroup SVD up to this LDS size (ACR_FUSED_LDS, bytes)
  bool svd_global = false;     // ACR_SVD_GLOBAL=1: every core takes the global-memory two-kernel path
  bool pchol_global = false;   // ACR_PCHOL_GLOBAL=1: every Gram takes the left-looking global-memory kernel
  bool inverse_unblocked = false;  // ACR_INVERSE_UNBLOCKED=1: unblocked Gauss-Jordan for every inverse
  bool pchol_lds = false;      // ACR_PCHOL_LDS=1: the right-looking LDS kernel instead of the register-tiled one
  bool pchol_512 = false;      // ACR_PCHOL_TILES=512: 512-thread 8 x 8 tiles for the whole large register-tiled kind
  bool pchol_mid = true;       // ACR_PCHOL_TILES=1024: orders 89-155 on 1024 threads too (else 512 threads, 5 x 5 tiles)
  bool gemm_narrow = true;     // ACR_GEMM_NARROW=0: FP32 outputs <= 32 columns wide in 64 x 64 tiles too
  bool svd_lq = true;          // ACR_SVD_LQ=0: cores too large for LDS keep W^T in the blocked global sweeps
  int merge_cus = 0;           // compute units for merging LDS size classes into one launch (ACR_NO_MERGE=1: 0, off)
  int leaf_lowp = 0;           // leaf x leaf products with 16-bit inputs: 1 = BF16, 2 = FP16 (FP32 data)
  int prod_lowp = 0;           // every factorisation product without its own choice, as leaf_lowp
  const char* trace_tag = "";
  void check_range(const void* p, size_t bytes, const char* what) const;

  // counters of launched algorithmic work (flops), by kernel class
  double flops_gemm = 0, flops_qr = 0, flops_svd = 0, flops_inv = 0;
  long launches = 0;

 private:
  struct Pending { hipEvent_t a, b; Work w; };
  std::vector<Pending> pending_;
  std::vector<hipEvent_t> event_pool_;
  unsigned long long* d_counters_ = nullptr;
  size_t counter_cursor_ = 0;
  std::vector<void*> oversized_;
  char* h_ring_ = nullptr;
  char* d_ring_ = nullptr;
  hipStream_t side_ = nullptr;    // second in-order stream for long independent stages
  hipEvent_t ev_[3] = {nullptr, nullptr, nullptr};
  size_t ring_bytes_ = 0, ring_off_ = 0;
};

// A low-rank block U V^T: U is rows x k, V is cols x k, both column-major.
template <class T> struct LR {
  T* U = nullptr;
  T* V = nullptr;
  int k = 0;
};

// Plane block: absent, diagonal, or HODLR (dense leaves + one low-rank block
// per off-diagonal position; block (d, s) has rows seg(d+1, s) and columns
// seg(d+1, s^1)).
template <class T> struct HMat {
  enum Kind { ABSENT = 0, DIAG = 1, HODLR = 2 };
  int kind = ABSENT;
  T* diag = nullptr;
  std::vector<T*> leaf;
  std::vector<LR<T>> blk;
  bool absent() const { return kind == ABSENT; }
  int max_rank() const {
    int m = 0;
    for (auto& b : blk) m = b.k > m ? b.k : m;
    return m;
  }
  size_t words(const Tree& tr) const;
};

// Truncation controls shared by all hierarchical operations.
struct Trunc {
  double eps = 0;         // stored blocks: keep sigma_i > eps * sigma_1
  double eps_inner = 0;   // internal accumulators of one operation
  int max_rank = 0;       // 0 = unlimited
};

// ---- hierarchical operations (batched over planes) ----
template <class T> struct MVJob {
  const HMat<T>* H;
  const std::vector<std::vector<LR<T>>>* corr;  // optional diagonal terms per depth
  const T* X;
  int64_t ldx;
  T* Y;
  int64_t ldy;
  int c;
  double alpha, beta;  // beta must be 0 or 1
};

template <class T> struct ProdJob {
  const HMat<T>* A;
  const HMat<T>* B;
  HMat<T>* C;
  double alpha;
};

template <class T> struct SumJob {
  std::vector<std::pair<const HMat<T>*, double>> terms;
  HMat<T>* C;
};

template <class T>
void hodlr_multivec(Exec& ex, const Tree& tr, const std::vector<MVJob<T>>& jobs, bool trans, int dmin,
                    Arena& scratch);
// `out` receives the result blocks; `work` holds intermediates for the duration
// of the call and `tmp` per-depth temporaries (both are rewound on return).
template <class T>
void hodlr_inverse(Exec& ex, const Tree& tr, const std::vector<const HMat<T>*>& D,
                   const std::vector<HMat<T>*>& G, const Trunc& tc, Arena& out, Arena& work, Arena& tmp);
template <class T>
void hodlr_product(Exec& ex, const Tree& tr, const std::vector<ProdJob<T>>& jobs, const Trunc& tc,
                   Arena& out, Arena& work, Arena& tmp);
template <class T>
void hodlr_sum(Exec& ex, const Tree& tr, const std::vector<SumJob<T>>& jobs, const Trunc& tc, Arena& out,
               Arena& tmp);
template <class T>
void hodlr_alloc_leaves(const Tree& tr, HMat<T>& H, Arena& out);

}  // namespace acr
