// bm_internal.hpp -- shared internal declarations of the Blind-Match GPU library.
//
// Data layout in HBM (all words uint64, residues in [0, q)):
//   polynomial          [limbs][N], limb-major, evaluation (NTT) domain in
//                        bit-reversed order unless stated otherwise
//   ciphertext          [comps][limbs][N]   (comps = 2, or 3 after a tensor)
//   ciphertext batch    [B][comps][limbs][N] with a per-batch element stride
//   switching key       [dnum][2][L+1+K][N] evaluation domain
//   gallery             [G][k][2][limbs][N]
// Limb l < L+1 is chain prime q_l; limb L+1+k is special prime p_k.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/blindmatch.h"

namespace bm {

using u64 = uint64_t;
using u32 = uint32_t;
using u128 = unsigned __int128;

constexpr int MAX_PRIMES = 24;   // chain + special primes
constexpr int MAX_LIMBS = 40;    // limb slots of one launch (all ModUp targets of a key switch)
constexpr int MAX_DIGITS = 16;
constexpr int MAX_ALPHA = 4;
// scratch of the no-allocation match, one array per device (see bm_match_noalloc)
constexpr size_t NOALLOC_SCRATCH_BYTES = BM_NOALLOC_SCRATCH_BYTES;

// ----------------------------------------------------------------- device runtime
//
// Every HIP runtime call of the library goes through these wrappers.  With
// the environment variable BM_DRY_RUN=1 they run without a GPU: device memory
// is host memory, copies are memcpy, kernel launches are skipped and every
// launch check still runs, so the launch geometry of whole call sequences can
// be validated on a CPU-only machine.
namespace dev {
bool dry();
hipError_t malloc_raw(void** p, size_t bytes);
template <class T>
inline hipError_t malloc(T** p, size_t bytes) { return malloc_raw((void**)p, bytes); }
hipError_t free(void* p);
hipError_t memcpy(void* d, const void* s, size_t bytes, hipMemcpyKind k);
hipError_t memcpy_async(void* d, const void* s, size_t bytes, hipMemcpyKind k, hipStream_t st);
hipError_t stream_sync(hipStream_t s);
hipError_t device_sync();
hipError_t stream_create(hipStream_t* s);
hipError_t stream_destroy(hipStream_t s);
hipError_t set_device(int d);
hipError_t event_create(hipEvent_t* e, bool timing);
hipError_t event_destroy(hipEvent_t e);
hipError_t event_record(hipEvent_t e, hipStream_t s);
hipError_t event_sync(hipEvent_t e);
hipError_t event_elapsed(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t event_query(hipEvent_t e);
hipError_t last_error();
hipError_t begin_capture(hipStream_t s);
hipError_t end_capture(hipStream_t s, hipGraph_t* g);
hipError_t graph_instantiate(hipGraphExec_t* e, hipGraph_t g);
hipError_t graph_destroy(hipGraph_t g);
hipError_t graph_launch(hipGraphExec_t e, hipStream_t s);
// Sizing pass of the calling thread: while a SizingScope is alive, kernel
// launches are skipped (their launch checks still run) and no other HIP call
// is made, so that a call sequence can be walked on the host to measure the
// scratch memory it needs before any of it is enqueued.
bool sizing();
struct SizingScope {
  SizingScope();
  ~SizingScope();
};
}  // namespace dev

// ----------------------------------------------------------------- errors

struct Error {
  int code;
  std::string msg;
};

#define BM_THROW(code, msg) throw ::bm::Error{(code), (msg)}
#define HIP_OK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      BM_THROW(BM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

// ----------------------------------------------------------------- per-prime constants (device)

struct PrimeC {
  u64 q;
  u64 qn;       // -q^{-1} mod 2^64 (Montgomery)
  u64 r2;       // 2^128 mod q
  u64 ninv;     // N^{-1} mod q
  u64 ninv_s;   // Shoup companion of ninv
  u64 pad[3];   // [0] floor(2^64 / q); [1] bits of the double 1/q; [2] bits of the double ninv/q
};

// Limb selection for one launch: limb slot y of every polynomial in the
// batch lives at element offset off[y]*N and belongs to prime prime[y].
struct LimbMap {
  int n;
  int prime[MAX_LIMBS];
  int off[MAX_LIMBS];    // input offset (limbs)
  int ooff[MAX_LIMBS];   // output offset (limbs); equal to off unless remapped
};

// ----------------------------------------------------------------- base-conversion tables (device)

struct ModUpDigit {
  int nsrc;                              // limbs of the digit present at this level
  int src[MAX_ALPHA];                    // their limb indices (= chain prime ids)
  u64 qhatinv[MAX_ALPHA][2];             // (Q_j/q_i)^{-1} mod q_i, Shoup pair
  u64 qhat[MAX_ALPHA][MAX_LIMBS][2];     // (Q_j/q_i) mod target slot t, Shoup pair
};

struct ModUpTable {                       // one per level (number of chain limbs)
  int limbs;                             // l
  int beta;                              // digits present
  int ext;                               // l + K target slots: chain limbs then specials
  int ext_prime[MAX_LIMBS];
  int npairs;                            // (digit, target slot outside the digit) pairs
  int8_t pair_j[MAX_LIMBS];
  int8_t pair_t[MAX_LIMBS];
  ModUpDigit d[MAX_DIGITS];
};

// Galois elements of a hoisted rotation sum, passed by value to the kernels:
// g[a] for amount a of every element, or g[(z % mod) * A + a] per element z
// (mod = the elements of one amount list, e.g. the k parts of each query).
constexpr int HOIST_MAX = 256;
struct HoistArgs {
  uint32_t g[HOIST_MAX];
  int A;
  int per_elem;
  int mod = 1 << 30;
};

// Per-element operand addresses of one launch, passed by value: element z of
// a launch reads or writes at p[z].  A launch covers at most PTR_MAX elements.
constexpr int PTR_MAX = 64;
struct PtrTab {
  const u64* p[PTR_MAX];
};
struct OutTab {
  u64* p[PTR_MAX];
};

struct ModDownTable {
  int K;
  int pprime[4];                          // prime ids of the special primes
  u64 phatinv[4][2];                      // (P/p_k)^{-1} mod p_k
  u64 phat[4][MAX_PRIMES][2];             // (P/p_k) mod q_i
  u64 pinv[MAX_PRIMES][2];                // P^{-1} mod q_i
};

// Work folded into the two passes of a forward transform at N = 2^16 (see
// kern::ntt_fused).  The column pass computes its input words on the fly from
// coefficient-domain sources (prologue), the row pass finishes each output
// word against a second operand before storing it (epilogue).  With isrc the
// sources hold only the row pass of their inverse transform: the column pass
// finishes it on each source tile before the conversion.
// Batch element z of a source / minuend / output sits at
//   base + (z / div) * hi + (z % div) * lo + limb * N.
struct FuseArgs {
  int pro = 0;   // 1: ModUp digit conversion (pair slots of the ModUpTable),
                 // 2: ModDown conversion of the special limbs, 3: reduction of one limb,
                 // 4: relinearisation and rescale in one (ModDown conversion of the
                 //    special limbs, the last chain limb reduced alongside)
  int epi = 0;   // 1: out = (minuend - x) w (+ addend) with w = wtab[2 slot];
                 // 2: out = (minuend wm + addend - x) w with wm = wmtab[2 slot]
  const ModUpTable* mu = nullptr;
  const ModDownTable* md = nullptr;
  const u64* src = nullptr;
  size_t s_hi = 0, s_lo = 0;
  int s_div = 1;
  int s_off0 = 0;                // ModDown: limb offset of the first special limb
  const u64* mnd = nullptr;
  size_t m_hi = 0, m_lo = 0;
  const u64* add0 = nullptr;     // addend of elements with z % div == 0
  size_t a0_hi = 0;
  const u64* add1 = nullptr;     // and of the others
  size_t a1_hi = 0;
  u64* out = nullptr;
  size_t o_hi = 0, o_lo = 0;
  int e_div = 1;
  const u64* wtab = nullptr;
  const u64* ci = nullptr;       // conjugate-invariant ring: the per-prime fold constants
  int src_pid = -1;              // one-limb reduction: prime of the source limb
  int last_off = -1;             // pro 4: limb offset (in a source component) of the last chain limb
  int last_pid = -1;             // pro 4: its prime
  const u64* wmtab = nullptr;    // epi 2: minuend multipliers
  int no_row = 0;                // 1: the column pass only (its words left in tmp)
  int isrc = 0;                  // 1: sources still need their inverse column pass
  const double* itwf = nullptr;  // isrc: inverse twiddles and their quotients w / q
  const double* itwq = nullptr;
  // epilogue output by reference: the base address is read from device
  // memory at *out_ref when the kernel runs, the output at base + out_rel
  // (out itself then only sizes the launch checks)
  u64* const* out_ref = nullptr;
  size_t out_rel = 0;
};

// ----------------------------------------------------------------- device memory

// Registry of live device allocations.  Every kernel launcher checks, before
// the launch, that each range its kernel will read or write lies inside one
// registered allocation, and raises BM_EINVAL instead of launching otherwise.
namespace audit {
void add(const void* p, size_t bytes);
void remove(const void* p);
// throws unless [p, p + bytes) is inside one registered allocation
void check(const void* p, size_t bytes, const char* what);
// RAII registration of a caller-owned buffer for the duration of a call
struct Scoped {
  const void* p;
  Scoped(const void* p_, size_t bytes) : p(p_) { add(p_, bytes); }
  ~Scoped() { remove(p); }
};
}  // namespace audit

// A caller's device allocator (bm_ctx_set_allocator).
struct AllocHook {
  void* (*alloc)(size_t bytes, void* user) = nullptr;
  void (*free)(void* p, void* user) = nullptr;
  void* user = nullptr;
};

// Caching allocator: blocks are recycled by exact size.  All work of a context
// is ordered on one stream, so a block freed by the host can be handed to the
// next request immediately (stream order protects pending readers).  New
// blocks come from the hook when one is set, else from hipMalloc; each block
// goes back to the allocator it came from, after a device synchronisation
// when that is the hook (hipFree synchronises by itself).
class DevicePool {
 public:
  explicit DevicePool(int device, std::shared_ptr<const AllocHook> hook = nullptr)
      : device_(device), hook_(std::move(hook)) {}
  // Arena mode: every block is carved out of [base, base + bytes), a region
  // the pool does not own (first fit, 256-byte aligned, freed ranges merged);
  // nothing is ever allocated from HIP or a hook.  An allocation that does not
  // fit raises BM_ENOMEM.  peak() is the highest end offset handed out.
  DevicePool(int device, void* base, size_t bytes);
  ~DevicePool();
  void* alloc(size_t bytes);
  void release(void* p, size_t bytes);
  size_t bytes_held() const { return held_; }
  // of which cached (freed, kept for reuse)
  size_t bytes_cached() const { return cached_; }
  size_t peak() const { return peak_; }
  void trim();
  // later blocks come from `hook` (null: hipMalloc); cached blocks are freed
  void set_hook(std::shared_ptr<const AllocHook> hook);

 private:
  void* new_block(size_t bytes);
  void free_cached();   // caller holds mu_
  void* arena_alloc(size_t bytes);
  void arena_release(void* p, size_t bytes);
  char* arena_ = nullptr;                 // arena mode when set
  size_t arena_bytes_ = 0, peak_ = 0;
  std::map<size_t, size_t> arena_free_;   // offset -> length of the free ranges
  int device_;
  std::shared_ptr<const AllocHook> hook_;
  std::map<void*, std::shared_ptr<const AllocHook>> hooked_;   // block -> the hook that made it
  std::multimap<size_t, void*> free_;
  size_t held_ = 0, cached_ = 0;
  std::mutex mu_;
};

struct Ctx;

// Optional per-kernel timing: when on, every kernel is launched with a pair of
// HIP events that the runtime stamps with the kernel's own start and end, and
// is charged with its algorithmic bytes and operations (counted by the
// launcher from the shapes it was given).
class Profiler {
 public:
  struct Entry {
    uint64_t launches = 0;
    double ms = 0, bytes = 0, ops = 0;
  };
  bool on = false;
  // events for the next launch, charged to `name`
  std::pair<hipEvent_t, hipEvent_t> begin(const char* name, double bytes, double ops);
  void collect();                       // waits for pending events, accumulates
  void reset();
  std::map<std::string, Entry> entries;
  ~Profiler();

 private:
  struct Pending {
    std::string name;
    hipEvent_t a, b;
    double bytes, ops;
  };
  std::vector<Pending> pending_;
  std::vector<hipEvent_t> spare_;
  std::mutex mu_;
  hipEvent_t take();
};

// RAII device buffer of u64 words from the context's current pool; it goes
// back to the pool it came from (a graph's private pool during a capture) and
// keeps that pool alive, so a buffer may outlive the context or server lane
// that made it.
class DBuf {
 public:
  DBuf() = default;
  DBuf(Ctx* c, size_t words);
  ~DBuf();
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept;
  u64* p() const { return p_; }
  size_t words() const { return words_; }

 private:
  std::shared_ptr<DevicePool> pool_;
  u64* p_ = nullptr;
  size_t words_ = 0;
};

// A captured match: replayed with the query copied into q_slot and the
// result copied out of out_slot.  Its scratch lives in its own pool.
struct GraphEntry {
  std::vector<uint64_t> key;
  std::shared_ptr<DevicePool> pool;
  DBuf q_slot, out_slot;
  DBuf out_ref;              // one device word: the replay's output base (by_ref)
  bool by_ref = false;       // the graph writes its output at *out_ref, not out_slot
  std::vector<DBuf> slots;   // a batch's query slots, one per shape class
  hipGraphExec_t exec = nullptr;
  ~GraphEntry();
};

// ----------------------------------------------------------------- context

struct HostPrime {
  u64 q;
  int bits;
  u64 psi;                 // primitive M-th root used by the device NTT (2N, or 4N: conjugate-invariant)
};

struct Ctx {
  int device = 0;
  int log_n = 0;
  size_t N = 0, n = 0;     // ring dimension and slots (N/2, or N in the conjugate-invariant ring)
  bool ci = false;         // conjugate-invariant ring R' = Z[X + X^-1] of rank N
  u64 M = 0;               // order of the roots behind the slots: 2N, or 4N in the conjugate-invariant ring
  int L = 0;               // top level; fresh ciphertexts have L+1 limbs
  int K = 0, alpha = 1, dnum = 1;
  double scale = 0, sigma = 3.2;
  uint32_t out_limbs = 0;  // default output limbs of a match (0 = natural level)
  std::vector<HostPrime> primes;   // L+1 chain primes then K special primes
  std::vector<u64> cdt;            // Gaussian cumulative table (38 entries)
  hipStream_t stream = nullptr;    // current stream of this context
  hipStream_t own_stream = nullptr;
  std::shared_ptr<DevicePool> pool;
  std::shared_ptr<const AllocHook> hook;   // caller's allocator for pools made from now on
  // device tables
  PrimeC* d_primes = nullptr;
  u64* d_tw = nullptr;             // [MAX_PRIMES][N] psi^{brv(k)} and Shoup companions
  u64* d_tws = nullptr;
  u64* d_itw = nullptr;            // psi^{-brv(k)}
  u64* d_itws = nullptr;
  double* d_twf = nullptr;         // the same twiddles as doubles, and w / q rounded (FP64 NTT)
  double* d_twq = nullptr;
  double* d_itwf = nullptr;
  double* d_itwq = nullptr;
  u64* d_ci = nullptr;             // conjugate-invariant ring: [MAX_PRIMES][4] iota = zeta^N, its Shoup
                                   // companion, 1/2 and its companion (the fold to Z_q[X]/(X^N - iota))
  ModUpTable* d_modup = nullptr;   // [L+2] indexed by number of chain limbs
  ModDownTable* d_moddown = nullptr;
  u64* d_rescale = nullptr;        // [L+1][L+1][2]: q_l^{-1} mod q_i, Shoup pair
  std::vector<ModUpTable> h_modup;
  ModDownTable h_moddown{};
  std::string last_error;
  // tuning knobs (result-invariant)
  int group_chunk = 0;             // gallery groups per batched pass (0 = auto)
  int kip_variant = 0;             // hoisted key inner product: elements x amounts per thread (0 = default)
  int ntt_views = 0;               // row-pass views per block of the N = 2^16 transforms (0 = 16)
  int kip_order = 0;               // block order of the grouped hoisted key inner product (0 / 1)
  int fused_occ = 0;               // 4: fused column passes built for 4 resident blocks per CU
  int col_src = 0;                 // 1: sources' inverse column pass in a launch of its own

  bool owns_tables = true;         // false for a lane sharing another context's tables
  std::shared_ptr<Profiler> prof = std::make_shared<Profiler>();
  bool use_graphs = false;                          // capture and replay matches
  std::vector<std::unique_ptr<GraphEntry>> graphs;  // most recent last
  // while a match is captured: fused ModDown epilogues whose output lies in
  // [ref_base, ref_base + ref_words) write it through the device word
  // ref_dev instead (ref_hits counts them, ref_covered their output words)
  u64* const* ref_dev = nullptr;
  const u64* ref_base = nullptr;
  size_t ref_words = 0;
  int ref_hits = 0;
  size_t ref_covered = 0;   // output words those epilogues write

  int nprimes() const { return (int)primes.size(); }
  int pid_special(int k) const { return L + 1 + k; }
  // limbs of a mask plaintext: every prime (the masked hoisted expansion
  // reads the special ones)
  int mask_limbs() const { return L + 1 + K; }
  void use_stream(void* s);
  // A context sharing this one's parameters and device tables, with its own
  // stream and memory pool (work on it overlaps with work on this one).
  std::unique_ptr<Ctx> make_lane() const;
  ~Ctx();
};

// ----------------------------------------------------------------- host math (host_math.cpp)

u64 h_mulmod(u64 a, u64 b, u64 q);
u64 h_powmod(u64 b, u64 e, u64 q);
u64 h_invmod(u64 a, u64 q);
u64 h_shoup(u64 w, u64 q);
bool h_is_prime(u64 n);
u64 h_primitive_2n_root(u64 q, size_t N);
void build_context_tables(Ctx& c);
std::vector<u64> gaussian_cdt(double sigma, int bound);

// SHAKE-256 streams and samplers (shake.cpp)
void shake256(const uint8_t* in, size_t inlen, uint8_t* out, size_t outlen);
void sample_ternary(u64 seed, u32 domain, u64 index, size_t n, int64_t* out);
void sample_gauss(const Ctx& c, u64 seed, u32 domain, u64 index, size_t n, int64_t* out);
void sample_uniform(u64 seed, u32 domain, u64 index, const u64* qs, size_t nq, size_t n, u64* out);

// canonical-embedding encoder (encoder.cpp)
void encode_slots(size_t N, const double* re, const double* im, double scale, int64_t* out);
void decode_coeffs(size_t N, const double* m, double scale, double* re, double* im);
// the context's ring: n real slot values -> N integer coefficients, and back
// (conjugate-invariant ring: through Z[X]/(X^2N+1), see encoder.cpp)
void ring_encode(const Ctx& c, const double* slots, double scale, int64_t* out);
void ring_decode(const Ctx& c, const double* m, double scale, double* slots);

// ----------------------------------------------------------------- device kernels (kernels.hip)

namespace kern {
// device address of the no-allocation scratch array on `device` (the device is
// made current; looked up once per device, then cached)
void* noalloc_scratch(int device);
LimbMap chain_map(int limbs);                        // q_0..q_{limbs-1} at offsets 0..
LimbMap ext_map(const Ctx& c, int limbs);           // q_0..q_{l-1}, p_0..p_{K-1}
LimbMap single(int prime, int off);

// forward / inverse negacyclic NTT; in and out may alias.  In the
// conjugate-invariant ring `raw` leaves out the fold (forward) or unfold
// (inverse) around the transform.
void ntt(const Ctx& c, const u64* in, size_t in_stride, u64* out, size_t out_stride, int B,
         const LimbMap& m, bool inverse, bool raw = false);
// in place: residue words (< 2^52) <-> the bit patterns of the same values as
// FP64 numbers (the form switching keys are kept in)
void words_f64(const Ctx& c, u64* p, size_t n, bool to_f64);
// register-resident issue-rate probe of the FP64 butterfly (k_modmul_rate)
void modmul_rate(const Ctx& c, int pid, int blocks, int iters, const u64* seed, u64* out);
// whether ntt_fused serves this context (N = 2^16)
bool fused_ok(const Ctx& c);
// the row pass of the inverse transform at N = 2^16 only (the words a fused
// column pass with isrc takes as sources)
void ntt_inv_rows(const Ctx& c, const u64* in, size_t in_stride, u64* out, size_t out_stride, int B,
                  const LimbMap& m);
// the column pass of the inverse transform at N = 2^16 only (its input the
// row pass's output, as ntt_inv_rows leaves it)
void ntt_inv_cols(const Ctx& c, const u64* in, size_t in_stride, u64* out, size_t out_stride, int B,
                  const LimbMap& m);
// whether the fused column pass can finish the inverse transform of its
// sources itself (f.isrc) for prologue kind pro: N = 2^16, outside the
// conjugate-invariant ring, at most 5 source primes per block
bool isrc_ok(const Ctx& c, int pro);
// forward NTT of the words f's prologue computes, into tmp at the slots m.ooff
// (slot s of element z at tmp + z * ts + m.ooff[s] * N), as FP64 values when
// f64_out; with an epilogue the finished words go to f.out instead and tmp
// only carries the first pass
void ntt_fused(const Ctx& c, const FuseArgs& f, u64* tmp, size_t ts, int B, const LimbMap& m,
               bool f64_out = false);
// signed integer polynomial [N] -> residues in limbs of m (coefficient domain)
void reduce_int(const Ctx& c, const int64_t* src, u64* out, size_t out_stride, int B,
                size_t src_stride, const LimbMap& m);
// out[z][comp][l] = ct[z / ct_div][comp][l] * pt[z % pt_mod][l], both
// components, chain limbs l < limbs (ccs / ocs: component strides)
void mul_ct_pt(const Ctx& c, const u64* ct, size_t sct, size_t ccs, const u64* pt, size_t spt, u64* out, size_t so,
               size_t ocs, int B, int limbs, int ct_div = 1, int pt_mod = 1 << 30);
// out = a + b, a - b, a * b (general), per limb of m; strides per operand (0 = broadcast)
void add(const Ctx& c, const u64* a, size_t sa, const u64* b, size_t sb, u64* o, size_t so,
         int B, const LimbMap& m);
void sub(const Ctx& c, const u64* a, size_t sa, const u64* b, size_t sb, u64* o, size_t so,
         int B, const LimbMap& m);
void mul(const Ctx& c, const u64* a, size_t sa, const u64* b, size_t sb, u64* o, size_t so,
         int B, const LimbMap& m);
// o_limb += s_limb * scalar[limb] (scalar per limb slot, Shoup pair list)
void axpy_scalar(const Ctx& c, const u64* s, size_t ss, const u64* scal /*[n][2] device*/,
                 u64* o, size_t so, int B, const LimbMap& m);
// tensor products of n elements whose operands sit at a[z] and b[z] (host
// lists of device addresses; any n, split into launches of PTR_MAX): the
// same product and part sum as tensor() below, output o + z so
void tensor_ptrs(const Ctx& c, const u64* const* a, size_t a_cs, size_t a_ps, const u64* const* b, size_t b_cs,
                 size_t b_ps, int parts, u64* o, size_t so, int n, int limbs);
// out[z] (host list of device addresses) = `limbs` limbs of both components of
// in + z si (component strides ics and ocs)
void copy_ptrs(const Ctx& c, const u64* in, size_t si, size_t ics, u64* const* out, size_t ocs, int n,
               int comps, int limbs);
// tensor product (a0,a1) x (b0,b1) -> (d0,d1,d2), optionally accumulated into o;
// batch element z uses a[z / a_div] and b[z % b_mod]
// a_cs, b_cs: component strides of the operands (>= limbs * N); with parts > 1
// the tensors of parts pairs (a + p a_ps, b + p b_ps) are summed
void tensor(const Ctx& c, const u64* a, size_t sa, int a_div, size_t a_cs, const u64* b, size_t sb,
            int b_mod, size_t b_cs, u64* o, size_t so, int B, int limbs, bool accumulate, int parts = 1, size_t a_ps = 0,
            size_t b_ps = 0);
// evaluation-domain automorphism X -> X^g of `comps` components of `limbs` limbs
// batch element z uses Galois element g1 when bit `sel` of z is set, else g0
void automorphism(const Ctx& c, const u64* in, size_t si, u64* out, size_t so, int B,
                  int rows, u64 g0, u64 g1, int sel);
// ModUp of every digit: coefficient-domain x [l] -> y[j][t] for every target slot t
// outside digit j (coefficient domain); y is [beta][ext][N] per batch element
void modup(const Ctx& c, const u64* xc, size_t sx, u64* y, size_t sy, int B, int limbs);
// key inner product: u/w[t] = sum_j y[j][t] * key_j[t]   (y: [beta][ext])
// batch element z uses key1 when bit `sel` of z is set, else key0
// (dadd: P d added to the last chain limb of the outputs, see k_kip)
void kip(const Ctx& c, const u64* y, size_t sy, const u64* y_own, size_t sown, const u64* key0,
         const u64* key1, int sel, u64* uw, size_t suw, int B, int limbs, const u64* dadd = nullptr,
         size_t sd = 0, size_t dcs = 0);
// ModDown base conversion: special limbs of u (coefficient) -> conv [l] (coefficient)
void moddown_conv(const Ctx& c, const u64* uw, size_t suw, u64* conv, size_t sc, int B, int limbs);
// out = (u - conv) * P^{-1} (+ addend), both components
void moddown_finish(const Ctx& c, const u64* uw, size_t suw, const u64* conv, size_t sc,
                    const u64* add0, size_t sadd0, const u64* add1, size_t sadd1, u64* out,
                    size_t so, int B, int limbs);
// rescale: last limb (coefficient, comps polys) -> reduced copies for limbs 0..l-2
void rescale_conv(const Ctx& c, const u64* last, size_t sl, size_t last_comp_stride, u64* t,
                  size_t st, int B, int comps, int limbs);
void rescale_finish(const Ctx& c, const u64* in, size_t si, const u64* t, size_t st, u64* out,
                    size_t so, int B, int comps, int limbs);
// batch element z is written to out + (z / div) so_hi + (z % div) so_lo; with
// ref, the launch also stores ref_val at the device word ref
void copy_limbs(const Ctx& c, const u64* in, size_t si, size_t in_comp_stride, u64* out, int div,
                size_t so_hi, size_t so_lo, size_t out_comp_stride, int B, int comps, int limbs,
                u64** ref = nullptr, u64* ref_val = nullptr);
// out[0 .. words) = 0
void zero(const Ctx& c, u64* out, size_t words);
// B elements of `words` words: gather out[z] = in[idx[z]] or scatter
// out[idx[z]] = in[z]; idx_dev is a device array of B indices <= max_idx
void move_idx(const Ctx& c, const u64* in, size_t si, u64* out, size_t so, const uint32_t* idx_dev,
              uint32_t max_idx, bool scatter, int B, size_t words);
// (u, w)[z] = sum_a KIP(phi_{g(z,a)}(y[z]), key_{g(z,a)}); gtab[g/2] holds the
// key of element g; `keys` lists the keys used (launch check).  The same
// launch computes c0_out[z] = c0_in[z] + sum_a phi_{g(z,a)}(c0_in[z]) over
// `limbs` limbs (accumulate: both outputs are added to; c0_out must not alias
// c0_in).
// key inner product of a plain key switch on whole rows (k_kip_rows, N = 2^16,
// standard ring): y holds the ModUp column pass's words (u64, pair slots), the
// row pass of the digits, the products and (slots >= inv_from) the row pass of
// the inverse transform in one launch; otherwise as kip
void kip_rows(const Ctx& c, const u64* y, size_t sy, const u64* y_own, size_t sown, const u64* key0,
              const u64* key1, int sel, u64* uw, size_t suw, int B, int limbs, int inv_from,
              const u64* dadd = nullptr, size_t sd = 0, size_t dcs = 0);
// masked hoisted rotation sums of Alg. 1's parts (k_kip_hoist_mask): per
// element e = j k + i (part i of query j at x + j sx, c1 at + xcs) the key
// sums over Q_l u P to uw [E][2][l+K][N] (with dadd: P times the addends added
// at the last chain limb) and the addends to ad [E][2][limbs][N]; masks
// [k][L+1+K][N]; parts[i] lists part i's Galois elements (k = parts.size(),
// every list of one length).  inv_rows (with dadd): the last chain limb and
// the special limbs of (u, w) may leave in their inverse row pass (N = 2^16,
// standard ring); the return value says whether they did
bool kip_hoist_mask(const Ctx& c, const u64* y, size_t sy, const u64* x, size_t sx, size_t xcs,
                    const u64* const* gtab, const std::vector<std::vector<uint32_t>>& parts,
                    const std::vector<const u64*>& keys, const u64* masks, u64* uw, size_t suw, u64* ad,
                    size_t sad, int nq, int limbs, bool dadd, bool inv_rows);
// inv_special: the special limbs of (u, w) may leave in their inverse row
// pass (the grouped kernel at N = 2^16, a non-accumulating launch); the
// return value says whether they did
bool kip_hoist(const Ctx& c, const u64* y, size_t sy, const u64* y_own, size_t sown, const u64* const* gtab,
               const HoistArgs& h, const std::vector<const u64*>& keys, u64* uw, size_t suw, const u64* c0_in,
               size_t c0_si, u64* c0_out, size_t c0_so, int B, int limbs, bool accumulate, bool inv_special);
}  // namespace kern

}  // namespace bm

// ----------------------------------------------------------------- opaque handles

struct bm_ct {
  bm_ctx* ctx = nullptr;
  bm::DBuf buf;            // [comps][limbs][N], evaluation domain
  uint32_t comps = 2, limbs = 0;
  double scale = 1.0;
  uint32_t query_d = 0;    // d of a bm_encrypt_query packing; 0 when not known
};

struct bm_sk {
  bm_ctx* ctx = nullptr;
  std::vector<int64_t> s;  // ternary coefficients
  bm::DBuf s_ntt;          // [L+1+K][N] evaluation domain
};

struct bm_pk {
  bm_ctx* ctx = nullptr;
  bm::DBuf pk;             // [2][L+1][N] evaluation domain (b, a)
};

struct bm_switch_key {
  bm::DBuf k;              // [dnum][2][L+1+K][N] evaluation domain
};

struct bm_evk {
  bm_ctx* ctx = nullptr;
  bm_switch_key rlk;
  std::map<uint64_t, std::unique_ptr<bm_switch_key>> gk;   // by Galois element
  bm::DBuf gtab;           // [N] device addresses of the Galois keys, at g / 2 (0 if absent)
};

struct bm_masks {
  bm_ctx* ctx = nullptr;
  uint32_t d = 0, k = 0;
  double scale = 0;
  bm::DBuf pt;             // [k][L+1+K][N] evaluation domain, every prime
};

struct bm_ctx {
  bm_params params;        // as created
  bm::Ctx c;
  // masks of Alg. 1 per (d, k), made on first use (declared after c: freed first)
  std::map<uint64_t, std::unique_ptr<bm_masks>> mask_cache;
};

struct bm_gallery {
  bm_ctx* ctx = nullptr;
  uint32_t d = 0, k = 0, limbs = 0;
  uint64_t n_templates = 0, groups = 0;
  double scale = 0;
  bm::DBuf buf;            // [G][k][2][limbs][N]
};

struct bm_result {
  bm_ctx* ctx = nullptr;
  uint32_t d = 0, k = 0, limbs = 0;
  uint64_t n_templates = 0, groups = 0;   // groups = result ciphertexts
  uint32_t packed = 0;                      // groups per ciphertext when compressed, else 0
  double scale = 0;
  std::shared_ptr<bm::DBuf> store;   // may be shared by the results of one batch
  size_t off = 0;                     // words; this result is [G][2][limbs][N] at store + off
  uint64_t* p() const { return store->p() + off; }
};
