// ckr_lib.cpp -- context, device pool, evaluator, key generation, circuits and
// the C ABI of the ckr library.
//
// Every homomorphic step runs in the HIP kernels of ckr_kernels.hip on the
// context stream; the host only derives parameters, samples randomness,
// encodes plaintexts and sequences launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <unordered_set>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <atomic>
#include <set>
#include <functional>
#include <vector>

#include "../../include/ckr.h"
#include "host_math.h"
#include "internal.h"

namespace ckr {

#define HIPCHK_NOTHROW(x) (void)(x)
#define HIPCHK(x)                                                                               \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) throw Error{CKR_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
    } while (0)

static thread_local std::string g_last_error;

// ------------------------------------------------------------------------
// device memory pool with an HBM budget
// ------------------------------------------------------------------------
class Pool {
  public:
    void *(*ualloc)(size_t, void *) = nullptr;
    void (*ufree)(void *, void *) = nullptr;
    void *user = nullptr;
    size_t budget = 0, in_use = 0, held = 0, high = 0;

    // size classes: 64 KiB granules up to 1 MiB, then 8 classes per power of
    // two (at most 12.5% over), so blocks of nearby sizes serve each other
    static size_t round(size_t b) {
        if (b <= (size_t(1) << 20)) return (b + 65535) & ~size_t(65535);
        int e = 63 - __builtin_clzll((unsigned long long)(b - 1));
        const size_t g = size_t(1) << (e - 3);
        return (b + g - 1) & ~(g - 1);
    }

    // While an arena is set (the allocation-free entry point), every block
    // comes from it by bumping an offset: nothing is taken from the cache or
    // the allocator, nothing is returned to them, and the byte counts do not
    // move.  Blocks are released all at once by clear_arena().
    void set_arena(void *base, size_t bytes) {
        std::lock_guard<std::recursive_mutex> g(pmu_);
        arena_ = (char *)base;
        arena_size_ = bytes;
        arena_off_ = 0;
    }
    void clear_arena() {
        std::lock_guard<std::recursive_mutex> g(pmu_);
        arena_ = nullptr;
        arena_size_ = arena_off_ = 0;
    }

    // While a graph is being captured, every block the capture obtains is
    // tracked; blocks freed during the capture are reused only by the capture
    // and then handed to the graph (its replays write them).
    void begin_capture() {
        capturing_ = true;
        cap_set_.clear();
        cap_free_.clear();
    }
    std::vector<std::pair<void *, size_t>> end_capture() {
        std::lock_guard<std::recursive_mutex> g(pmu_);
        // every block the capture handed out and got back is the plan's,
        // whichever free list it sits on
        std::vector<const void *> streams;
        for (auto &st : sfree_) streams.push_back(st.first);
        for (const void *st : streams) take_captured_locked(st);
        capturing_ = false;
        std::vector<std::pair<void *, size_t>> owned;
        for (auto &kv : cap_free_)
            for (void *p : kv.second) owned.push_back({p, kv.first});
        cap_free_.clear();
        cap_set_.clear();
        return owned;
    }
    void release_owned(const std::vector<std::pair<void *, size_t>> &owned) {
        std::lock_guard<std::recursive_mutex> g(pmu_);
        for (auto &b : owned) cache_[b.second].push_back(b.first);
    }

    // Stream-local reuse.  While branches of one circuit run on several streams
    // (fork()..join()), or while a server issues batches on several slot
    // streams of this context (set_local), a freed block goes to a free list of
    // the stream that freed it and is reused only by later allocations on that
    // same stream (stream order makes that safe); blocks freed before serve
    // every stream.  A join moves the branches' lists to the joining stream,
    // whose wait orders every branch before its later work (or, with no server,
    // returns every list to the common cache); flush(stream), called once the
    // host has waited for that stream, returns its list to the common cache.
    // Blocks a graph capture uses stay the capture's (cap_free_) either way.
    // `cur` names the stream work is being issued on.
    void set_cur(const void *const *cur) { cur_ = cur; }
    void set_local(bool on) {
        std::lock_guard<std::recursive_mutex> g(pmu_);
        local_ += on ? 1 : -1;
        if (local_ == 0 && forked_ == 0) release_all_locked();
    }
    void fork() {
        std::lock_guard<std::recursive_mutex> g(pmu_);
        forked_++;
    }
    void join(const void *main, const void *const *sides, int nsides) {
        std::lock_guard<std::recursive_mutex> g(pmu_);
        --forked_;
        if (local_ == 0 && forked_ == 0) {
            release_all_locked();
            return;
        }
        for (int i = 0; i < nsides; i++) {
            if (sides[i] == main) continue;
            auto st = sfree_.find(sides[i]);
            if (st == sfree_.end()) continue;
            for (auto &kv : st->second)
                for (void *p : kv.second) {
                    if (capturing_ && cap_set_.count(p)) cap_free_[kv.first].push_back(p);
                    else sfree_[main][kv.first].push_back(p);
                }
            sfree_.erase(sides[i]);
        }
        // Blocks of a capture freed on the joining stream while the branches
        // were open belong to the capture as well: everything captured after
        // the join is ordered after it, so they go back to the capture's free
        // list.  Left in the stream's list they would outlive end_capture()
        // and be handed to other work while the graph's replays still use them.
        if (capturing_) take_captured_locked(main);
    }
    // capture-owned blocks of `stream`'s free list -> cap_free_
    void take_captured_locked(const void *stream) {
        auto st = sfree_.find(stream);
        if (st == sfree_.end()) return;
        for (auto &kv : st->second) {
            auto &v = kv.second;
            for (size_t i = 0; i < v.size();) {
                if (cap_set_.count(v[i])) {
                    cap_free_[kv.first].push_back(v[i]);
                    v[i] = v.back();
                    v.pop_back();
                } else {
                    i++;
                }
            }
        }
    }
    void flush(const void *stream) {
        std::lock_guard<std::recursive_mutex> g(pmu_);
        auto st = sfree_.find(stream);
        if (st == sfree_.end()) return;
        for (auto &kv : st->second)
            for (void *p : kv.second) release_locked(p, kv.first);
        sfree_.erase(st);
    }

    void *get(size_t bytes) {
        std::lock_guard<std::recursive_mutex> g(pmu_);
        if (arena_) {
            const size_t off = (arena_off_ + 255) & ~size_t(255);
            if (off + bytes > arena_size_) throw Error{CKR_E_NOMEM, "scratch exhausted"};
            arena_off_ = off + bytes;
            return arena_ + off;
        }
        bytes = round(bytes);
        if (capturing_) {
            auto cf = cap_free_.find(bytes);
            if (cf != cap_free_.end() && !cf->second.empty()) {
                void *p = cf->second.back();
                cf->second.pop_back();
                in_use += bytes;
                high = std::max(high, in_use);
                return p;
            }
        }
        void *p = nullptr;
        if (forked_ || local_) {
            auto st = sfree_.find(*cur_);
            if (st != sfree_.end()) {
                auto it = st->second.find(bytes);
                if (it != st->second.end() && !it->second.empty()) {
                    p = it->second.back();
                    it->second.pop_back();
                    in_use += bytes;
                    high = std::max(high, in_use);
                }
            }
        }
        if (!p) p = get_uncaptured(bytes);
        if (capturing_) cap_set_.insert(p);
        return p;
    }

    void *get_uncaptured(size_t bytes) {
        auto it = cache_.find(bytes);
        if (it != cache_.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            in_use += bytes;
            high = std::max(high, in_use);
            return p;
        }
        if (budget && held + bytes > budget && !capturing_) trim();
        if (budget && held + bytes > budget) throw Error{CKR_E_NOMEM, "HBM budget exceeded"};
        void *p = nullptr;
        if (ualloc) {
            p = ualloc(bytes, user);
        } else if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            // out of device memory: return cached blocks to the device, the
            // largest first, only until the allocation fits (freeing the whole
            // cache would make every later block a fresh allocation)
            if (!capturing_) p = evict_for(bytes);
        }
        if (!p) throw Error{CKR_E_NOMEM, "device allocation failed"};
        held += bytes;
        in_use += bytes;
        high = std::max(high, in_use);
        return p;
    }
    void put(void *p, size_t bytes) {
        if (!p) return;
        std::lock_guard<std::recursive_mutex> g(pmu_);
        if (arena_ && (char *)p >= arena_ && (char *)p < arena_ + arena_size_) return;
        bytes = round(bytes);
        in_use -= bytes;
        if (forked_ || (local_ && !(capturing_ && cap_set_.count(p)))) {
            sfree_[*cur_][bytes].push_back(p);
            return;
        }
        release_locked(p, bytes);
    }
    void *evict_for(size_t bytes) {
        std::vector<size_t> sizes;
        for (auto &kv : cache_)
            if (!kv.second.empty()) sizes.push_back(kv.first);
        std::sort(sizes.rbegin(), sizes.rend());
        size_t freed = 0;
        for (size_t sz : sizes) {
            auto &v = cache_[sz];
            while (!v.empty()) {
                (void)hipFree(v.back());
                v.pop_back();
                held -= sz;
                freed += sz;
                if (freed >= bytes) {
                    void *p = nullptr;
                    if (hipMalloc(&p, bytes) == hipSuccess) return p;
                    (void)hipGetLastError();
                    freed = 0;
                }
            }
        }
        void *p = nullptr;
        if (hipMalloc(&p, bytes) == hipSuccess) return p;
        (void)hipGetLastError();
        return nullptr;
    }
    // return cached blocks to the allocator (stream-ordered frees are safe
    // because the caller synchronises first)
    void trim() {
        std::lock_guard<std::recursive_mutex> g(pmu_);
        for (auto &kv : cache_) {
            for (void *p : kv.second) {
                if (ufree) ufree(p, user);
                else (void)hipFree(p);
                held -= kv.first;
            }
            kv.second.clear();
        }
    }
    ~Pool() {
        release_all_locked();
        trim();
    }

  private:
    void release_locked(void *p, size_t bytes) {
        if (capturing_ && cap_set_.count(p)) cap_free_[bytes].push_back(p);
        else cache_[bytes].push_back(p);
    }
    void release_all_locked() {
        for (auto &st : sfree_)
            for (auto &kv : st.second)
                for (void *p : kv.second) release_locked(p, kv.first);
        sfree_.clear();
    }
    std::recursive_mutex pmu_;
    int forked_ = 0, local_ = 0;
    const void *const *cur_ = nullptr;
    std::map<const void *, std::unordered_map<size_t, std::vector<void *>>> sfree_;
    std::unordered_map<size_t, std::vector<void *>> cache_;
    bool capturing_ = false;
    std::unordered_set<void *> cap_set_;
    std::unordered_map<size_t, std::vector<void *>> cap_free_;
    char *arena_ = nullptr;
    size_t arena_size_ = 0, arena_off_ = 0;
};

struct Ctx;

// RAII device buffer drawn from the context pool
class Buf {
  public:
    Buf() = default;
    Buf(Ctx *c, size_t words);
    Buf(Buf &&o) noexcept : c_(o.c_), p_(o.p_), words_(o.words_) { o.p_ = nullptr; }
    Buf &operator=(Buf &&o) noexcept {
        if (this != &o) {
            release();
            c_ = o.c_; p_ = o.p_; words_ = o.words_;
            o.p_ = nullptr;
        }
        return *this;
    }
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
    ~Buf() { release(); }
    u64 *get() const { return p_; }
    size_t words() const { return words_; }

  private:
    void release();
    Ctx *c_ = nullptr;
    u64 *p_ = nullptr;
    size_t words_ = 0;
};

// B ciphertexts at one level, layout [B][2][level+1][n]
struct DCt {
    int level = -1;
    int B = 0;
    Buf buf;
    u64 *d() const { return buf.get(); }
};

struct PlainKey {
    int kind, N, level, arg;
    bool operator<(const PlainKey &o) const {
        return std::tie(kind, N, level, arg) < std::tie(o.kind, o.N, o.level, o.arg);
    }
};

enum ProfCat {
    kNttFwdCol, kNttFwdRow, kNttInvRow, kNttInvCol, kBConv, kNttRowIP, kTensor, kAutomorph, kElem, kCopy, kNCat
};
static const char *kCatName[kNCat] = {"ntt_fwd_col", "ntt_fwd_row", "ntt_inv_row", "ntt_inv_col", "bconv",
                                      "ntt_row_ip", "tensor", "automorph", "elementwise", "copy"};

// opt-in per-category kernel timing with HIP events on the context stream
struct Prof {
    bool on = false;
    struct Rec {
        int cat;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> spare;
    u64 launches[kNCat] = {};
    double ms[kNCat] = {}, bytes[kNCat] = {};
};

struct Ctx {
    Prof prof;
    bool graphs = true;           // capture batched circuits into hipGraphs
    int ntt_chunk = 0;            // limbs per two-pass chunk (0: whole dispatch), keeps pass-1 output in cache
    unsigned tune_epoch = 0;      // bumped by every tile or chunk change: older captured plans are re-captured
    hipStream_t own_stream = nullptr;
    static constexpr int kSide = 4;
    static constexpr int kSlots = 2;  // server slots: batches of one context in flight at once
    // slot 0: the API calls (stream = own_stream or the caller's); slots 1..kSlots: server batches
    int slot = 0;
    hipStream_t slot_stream[kSlots + 1] = {};
    hipStream_t side[kSlots + 1][kSide] = {};  // streams of concurrent circuit branches, per slot
    int forks = 0;                             // open Branches (at most one: they do not nest)
    // streams of server slot s (made on first use, default priority)
    void ensure_slot(int s) {
        if (slot_stream[s]) return;
        hipStream_t st = nullptr;
        if (hipStreamCreate(&st) != hipSuccess) throw Error{CKR_E_DEVICE, "slot stream"};
        slot_stream[s] = st;
        for (hipStream_t &x : side[s])
            if (!x && hipStreamCreate(&x) != hipSuccess) throw Error{CKR_E_DEVICE, "slot side stream"};
    }
    Params P;
    DevTables T{};
    hipStream_t stream = nullptr;
    int device = 0;
    u64 *scratch = nullptr;  // this device's copy of the allocation-free entry point's scratch array
    Pool pool;
    std::vector<void *> table_mem;  // owned by the context (tables)
    std::map<std::pair<int, int>, BConvTab> modup;  // (level, digit)
    std::map<int, BConvTab> moddown;                // level
    std::map<PlainKey, Buf> plain;                  // encoded plaintexts, eval domain
    std::map<std::vector<u64>, Buf> lincomb;        // Chebyshev linear-combination constants
    std::mutex mu;
    std::recursive_mutex mu_run;  // held while enqueueing work: API calls vs. server workers
    size_t n() const { return P.n; }

    void *table_alloc(size_t bytes) {
        void *p = nullptr;
        HIPCHK(hipMalloc(&p, bytes));
        table_mem.push_back(p);
        return p;
    }
    ~Ctx() {
        plain.clear();
        (void)hipDeviceSynchronize();  // every stream of the context (slots and branches) is done
        for (auto &r : prof.pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (hipEvent_t e : prof.spare) (void)hipEventDestroy(e);
        pool.trim();
        for (void *p : table_mem) (void)hipFree(p);
        if (own_stream) (void)hipStreamDestroy(own_stream);
        for (auto &row : side)
            for (hipStream_t st : row)
                if (st) (void)hipStreamDestroy(st);
        for (int i = 1; i <= kSlots; i++)
            if (slot_stream[i]) (void)hipStreamDestroy(slot_stream[i]);
    }
};

Buf::Buf(Ctx *c, size_t words) : c_(c), words_(words) { p_ = (u64 *)c->pool.get(words * 8); }
void Buf::release() {
    if (p_ && c_) c_->pool.put(p_, words_ * 8);
    p_ = nullptr;
}

// a batched circuit captured once into a hipGraph and replayed: it reads a
// plan-owned input batch and writes plan-owned outputs
struct GraphPlan {
    Ctx *C = nullptr;
    hipStream_t stream = nullptr;  // the stream its replays run on
    std::vector<DCt> in;  // one input batch per query group
    std::vector<DCt> outs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<std::pair<void *, size_t>> owned;  // temporaries the replays write
    unsigned long long last_use = 0;               // Keys::plan_clock at its latest replay
    unsigned epoch = 0;                            // Ctx::tune_epoch at capture
    ~GraphPlan() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (C) C->pool.release_owned(owned);
    }
};

// one circuit: kind (rank, order statistic, sort), N, the order statistic's rank window
// and tie-correction flag, comparator and indicator compositions
struct Spec {
    int kind = 0, N = 0, k = 0, k_hi = 0, tie = 0;  // order statistics: the rank window [k, k_hi]
    ckr_sign cmp{0, 0, 0}, ind{0, 0, 0};
    auto tup() const {
        return std::make_tuple(kind, N, k, k_hi, tie, cmp.d_g, cmp.d_f, cmp.cheb, cmp.minimax, ind.d_g, ind.d_f,
                               ind.cheb, ind.minimax);
    }
};
// a group of B inputs of one level running one circuit
struct GroupKey {
    Spec s;
    int level = 0, B = 0;
    bool operator<(const GroupKey &o) const {
        return std::tuple_cat(s.tup(), std::make_tuple(level, B)) < std::tuple_cat(o.s.tup(), std::make_tuple(o.level, o.B));
    }
};
using PlanKey = std::vector<GroupKey>;

struct Keys {
    Ctx *C = nullptr;
    int lmax = 0;
    std::vector<i64> s;               // ternary secret, host only
    Buf pk;                           // [2][lmax+1][n] eval domain
    std::map<u32, Buf> swk;           // galois element (0 = relinearisation) -> [beta][2][Ek][n]
    std::set<PlanKey> warm;           // circuits run once eagerly (caches filled)
    // captured plans per (slot, circuit): each slot replays its own copy, so
    // batches of several server slots never share a plan's buffers
    std::map<std::pair<int, PlanKey>, std::unique_ptr<GraphPlan>> plans;  // destroyed before the keys they read
    unsigned long long plan_clock = 0;
    int Ek() const { return lmax + 1 + C->P.K; }
};

// ------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------
static inline size_t limb_words(const Ctx &C) { return C.P.n; }

static DCt ct_new(Ctx &C, int level, int B) {
    DCt c;
    c.level = level;
    c.B = B;
    c.buf = Buf(&C, (size_t)B * 2 * (level + 1) * C.n());
    return c;
}

// Concurrent branches of one circuit.  Each run() issues its work on one of
// the context's side streams, ordered after everything issued on the current
// stream before the Branches object was made; join() orders everything issued
// afterwards on the current stream after every branch.  Under graph capture
// the branches become parallel paths of the graph, forked from and joined back
// to the capturing stream.  Branches never nest: inside an open fork, run()
// issues its work inline on the current stream.  Blocks freed inside a branch
// are reused only within that branch until the join (Pool::fork).
class Branches {
  public:
    // While kernel timing is on, branches run inline too: concurrent kernels
    // would stretch each other's event-bracketed durations.
    explicit Branches(Ctx &C) : C_(C), main_(C.stream), nested_(C.forks > 0 || C.prof.on) {
        if (nested_) return;
        C_.forks++;
        HIPCHK(hipEventCreateWithFlags(&fork_, hipEventDisableTiming));
        HIPCHK(hipEventRecord(fork_, main_));
        C_.pool.fork();
    }
    Branches(const Branches &) = delete;
    Branches &operator=(const Branches &) = delete;
    template <class F>
    void run(F &&f) {
        if (nested_) {
            f();
            return;
        }
        hipStream_t st = C_.side[C_.slot][next_++ % Ctx::kSide];
        used_[std::min(next_, Ctx::kSide) - 1] = st;
        HIPCHK(hipStreamWaitEvent(st, fork_, 0));
        C_.stream = st;
        struct Back {
            Ctx &C;
            hipStream_t m;
            ~Back() { C.stream = m; }
        } back{C_, main_};
        f();
        hipEvent_t e = nullptr;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ends_.push_back(e);
        HIPCHK(hipEventRecord(e, st));
    }
    void join() {
        if (joined_ || nested_) return;
        joined_ = true;
        hipError_t err = hipSuccess;
        for (hipEvent_t e : ends_) {
            const hipError_t r = hipStreamWaitEvent(main_, e, 0);
            if (err == hipSuccess) err = r;
        }
        pool_join();
        C_.forks--;
        release();
        if (err != hipSuccess) throw Error{CKR_E_DEVICE, std::string("branch join: ") + hipGetErrorString(err)};
    }
    ~Branches() {
        if (!joined_ && !nested_) {
            joined_ = true;
            for (hipEvent_t e : ends_) (void)hipStreamWaitEvent(main_, e, 0);
            pool_join();
            C_.forks--;
            release();
        }
    }

  private:
    void pool_join() {
        const void *sides[Ctx::kSide];
        const int ns = std::min(next_, Ctx::kSide);
        for (int i = 0; i < ns; i++) sides[i] = used_[i];
        C_.pool.join(main_, sides, ns);
    }
    void release() {
        for (hipEvent_t e : ends_) (void)hipEventDestroy(e);
        ends_.clear();
        if (fork_) (void)hipEventDestroy(fork_);
        fork_ = nullptr;
    }
    Ctx &C_;
    hipStream_t main_;
    hipEvent_t fork_ = nullptr;
    std::vector<hipEvent_t> ends_;
    bool nested_;
    int next_ = 0;
    hipStream_t used_[Ctx::kSide] = {};
    bool joined_ = false;
};

static hipEvent_t prof_event(Ctx &C) {
    if (!C.prof.spare.empty()) {
        hipEvent_t e = C.prof.spare.back();
        C.prof.spare.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
}

// wait for the context stream; every block freed on it is then free for
// every stream
static void sync(Ctx &C) {
    HIPCHK(hipStreamSynchronize(C.stream));
    C.pool.flush(C.stream);
}

// run `launch` on the context stream; when profiling, bracket it with events
template <class F>
static void timed(Ctx &C, int cat, double bytes, F &&launch) {
    if (!C.prof.on) {
        launch();
        return;
    }
    hipEvent_t a = prof_event(C), b = prof_event(C);
    HIPCHK(hipEventRecord(a, C.stream));
    launch();
    HIPCHK(hipEventRecord(b, C.stream));
    C.prof.pending.push_back({cat, a, b, bytes});
}

static void prof_resolve(Ctx &C) {
    if (C.prof.pending.empty()) return;
    sync(C);
    for (auto &r : C.prof.pending) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        C.prof.launches[r.cat]++;
        C.prof.ms[r.cat] += ms;
        C.prof.bytes[r.cat] += r.bytes;
        C.prof.spare.push_back(r.a);
        C.prof.spare.push_back(r.b);
    }
    C.prof.pending.clear();
}

// Each pass reads and writes every limb once: 16 n bytes per limb.  Large
// dispatches run in chunks of whole polynomials so the second pass reads the
// first pass's output while it is still in the last-level cache.
template <class F>
static void for_chunks(Ctx &C, int limbs, int polys, F &&f) {
    int per = polys;
    if (C.ntt_chunk > 0 && limbs * polys > C.ntt_chunk) per = std::max(1, C.ntt_chunk / std::max(limbs, 1));
    for (int p0 = 0; p0 < polys; p0 += per) f(p0, std::min(per, polys - p0));
}

static void ntt(Ctx &C, u64 *base, int limbs, int polys, size_t stride, LimbMap map, bool inv,
                const u64 *src = nullptr, size_t src_stride = 0, u32 gal = 0) {
    for_chunks(C, limbs, polys, [&](int p0, int np) {
        LimbBatch b{base + (size_t)p0 * stride, limbs, np, stride, map};
        if (src) {
            b.src = src + (size_t)p0 * src_stride;
            b.src_stride = src_stride;
            b.gal = gal;
        }
        const double bytes = 16.0 * C.P.n * limbs * np;
        timed(C, inv ? kNttInvRow : kNttFwdCol, bytes, [&] { k_ntt_pass(C.T, b, inv, 0, C.stream); });
        timed(C, inv ? kNttInvCol : kNttFwdRow, bytes, [&] { k_ntt_pass(C.T, b, inv, 1, C.stream); });
    });
}

// the first (column) pass of the forward transform only
static void ntt_first(Ctx &C, u64 *base, int limbs, int polys, size_t stride, LimbMap map) {
    LimbBatch b{base, limbs, polys, stride, map};
    timed(C, kNttFwdCol, 16.0 * C.P.n * limbs * polys, [&] { k_ntt_pass(C.T, b, false, 0, C.stream); });
}

// the second (column) pass of the inverse transform only, on data that has had
// the row pass
static void intt_second(Ctx &C, u64 *base, int limbs, int polys, size_t stride, LimbMap map) {
    LimbBatch b{base, limbs, polys, stride, map};
    timed(C, kNttInvCol, 16.0 * C.P.n * limbs * polys, [&] { k_ntt_pass(C.T, b, true, 1, C.stream); });
}

// forward transform with the fused prologue / epilogue of NttFuse.  The
// epilogue addresses poly p = 2b + k, so chunks hold whole (b) pairs.
static void ntt_fused(Ctx &C, u64 *base, int limbs, int polys, size_t stride, LimbMap map, const NttFuse &f) {
    const double limb = 8.0 * C.P.n;
    int per = polys;
    if (C.ntt_chunk > 0 && limbs * polys > C.ntt_chunk) per = std::max(2, (C.ntt_chunk / std::max(limbs, 1)) & ~1);
    for (int p0 = 0; p0 < polys; p0 += per) {
        const int np = std::min(per, polys - p0);
        LimbBatch b{base + (size_t)p0 * stride, limbs, np, stride, map};
        NttFuse g = f;
        const size_t b0 = (size_t)(p0 >> 1);  // first batch entry of the chunk
        if (g.pro) g.src = f.src + (size_t)p0 * f.src_stride;
        if (g.src2) g.src2 = f.src2 + (size_t)p0 * f.src2_stride;
        if (g.epi) {
            g.out = f.out + b0 * f.out_stride;
            g.x = f.x + b0 * f.x_stride;
            if (g.add) g.add = f.add + b0 * f.add_stride;
            if (g.add2) g.add2 = f.add2 + b0 * f.add2_stride;
        }
        const double all = limb * limbs * np;
        const double b0b = g.pro ? limb * np + all + (g.src2 ? all : 0) : 2 * all;
        const double b1b = g.epi ? 3 * all + (g.add ? all * __builtin_popcount(g.add_mask) / 2 : 0) +
                                       (g.add2 ? all * __builtin_popcount(g.add2_mask) / 2 : 0)
                                 : 2 * all;
        timed(C, kNttFwdCol, b0b, [&] { k_ntt_fused(C.T, b, g, 0, C.stream); });
        timed(C, kNttFwdRow, b1b, [&] { k_ntt_fused(C.T, b, g, 1, C.stream); });
    }
}

// 2-D strided device copy: `rows` rows of `width` words
static void copy2d(Ctx &C, u64 *dst, size_t dpitch, const u64 *src, size_t spitch, size_t width, size_t rows) {
    HIPCHK(hipMemcpy2DAsync(dst, dpitch * 8, src, spitch * 8, width * 8, rows, hipMemcpyDeviceToDevice, C.stream));
}

static void scalars_of(const Ctx &C, i64 K, int limbs, LimbMap map, LimbScalars &s) {
    if (limbs > kMaxLimbArgs) throw Error{CKR_E_INVALID, "too many limbs"};
    for (int t = 0; t < limbs; t++) {
        const u64 q = C.P.mod[map(t)];
        const u64 v = hred(K, q);
        s.v[t] = (double)v;
        s.vq[t] = (double)v / (double)q;
    }
}

static void scalars_of_vals(const Ctx &C, const std::vector<u64> &vals, LimbScalars &s) {
    if ((int)vals.size() > kMaxLimbArgs) throw Error{CKR_E_INVALID, "too many limbs"};
    for (size_t t = 0; t < vals.size(); t++) {
        s.v[t] = (double)vals[t];
        s.vq[t] = (double)vals[t] / (double)C.P.mod[t];
    }
}

// ------------------------------------------------------------------------
// context setup: twiddle tables and constants
// ------------------------------------------------------------------------
static u64 brev(u64 x, int bits) {
    u64 r = 0;
    for (int i = 0; i < bits; i++) r |= ((x >> i) & 1) << (bits - 1 - i);
    return r;
}

static void setup_tables(Ctx &C) {
    const Params &P = C.P;
    const int nm = P.nmod();
    const u64 n = P.n;
    C.T.logn = P.logn;
    C.T.nmod = nm;
    std::vector<double2> mq(nm), last(2 * nm);
    std::vector<double> fwdq((size_t)nm * n), invq((size_t)nm * n);  // w/q (IEEE division)
    std::vector<u64> qi(nm);
    std::vector<u64> pw(n), ipw(n);
    for (int t = 0; t < nm; t++) {
        const u64 q = P.mod[t];
        const double dq = (double)q;
        mq[t] = make_double2(dq, 1.0 / dq);
        qi[t] = q;
        const u64 psi = P.psi[t], ipsi = hinv(psi, q);
        pw[0] = 1; ipw[0] = 1;
        for (u64 j = 1; j < n; j++) {
            pw[j] = hmul(pw[j - 1], psi, q);
            ipw[j] = hmul(ipw[j - 1], ipsi, q);
        }
        for (u64 i = 0; i < n; i++) {
            const u64 w = pw[brev(i, P.logn)], wi = ipw[brev(i, P.logn)];
            fwdq[(size_t)t * n + i] = (double)w / dq;
            invq[(size_t)t * n + i] = (double)wi / dq;
        }
        const u64 ninv = hinv(n % q, q);
        const u64 w1 = hmul(ipw[n / 2], ninv, q);
        last[2 * t] = make_double2((double)ninv, (double)ninv / dq);
        last[2 * t + 1] = make_double2((double)w1, (double)w1 / dq);
    }
    C.T.mq = (double2 *)C.table_alloc(nm * sizeof(double2));
    C.T.qi = (u64 *)C.table_alloc(nm * sizeof(u64));
    C.T.tw_last = (double2 *)C.table_alloc(last.size() * sizeof(double2));
    HIPCHK(hipMemcpy(C.T.mq, mq.data(), nm * sizeof(double2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(C.T.qi, qi.data(), nm * sizeof(u64), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(C.T.tw_last, last.data(), last.size() * sizeof(double2), hipMemcpyHostToDevice));
    C.T.twq_fwd = (double *)C.table_alloc(fwdq.size() * sizeof(double));
    C.T.twq_inv = (double *)C.table_alloc(invq.size() * sizeof(double));
    HIPCHK(hipMemcpy(C.T.twq_fwd, fwdq.data(), fwdq.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(C.T.twq_inv, invq.data(), invq.size() * sizeof(double), hipMemcpyHostToDevice));
}

// fast base conversion table from moduli src[] to moduli tgt[] (output slots given)
static BConvTab make_bconv(Ctx &C, const std::vector<int> &src, const std::vector<int> &tgt,
                           const std::vector<int> &slot, bool round = false) {
    if ((int)src.size() > kMaxBConvSrc || (int)tgt.size() > kMaxLimbArgs) throw Error{CKR_E_INVALID, "bconv size"};
    BConvTab tab{};
    tab.ns = (int)src.size();
    tab.nt = (int)tgt.size();
    std::vector<double2> hi(tab.ns), hm((size_t)tab.ns * tab.nt);
    for (int i = 0; i < tab.ns; i++) {
        tab.src_mod[i] = src[i];
        const u64 qi = C.P.mod[src[i]];
        u64 prod = 1 % qi;
        for (int k = 0; k < tab.ns; k++)
            if (k != i) prod = hmul(prod, C.P.mod[src[k]] % qi, qi);
        const u64 v = hinv(prod, qi);
        hi[i] = make_double2((double)v, (double)v / (double)qi);
        for (int j = 0; j < tab.nt; j++) {
            const u64 t = C.P.mod[tgt[j]];
            u64 h = 1 % t;
            for (int k = 0; k < tab.ns; k++)
                if (k != i) h = hmul(h, C.P.mod[src[k]] % t, t);
            hm[(size_t)i * tab.nt + j] = make_double2((double)h, (double)h / (double)t);
        }
    }
    for (int j = 0; j < tab.nt; j++) {
        tab.tgt_mod[j] = tgt[j];
        tab.tgt_slot[j] = slot[j];
    }
    tab.hinv = (double2 *)C.table_alloc(hi.size() * sizeof(double2));
    tab.hmod = (double2 *)C.table_alloc(hm.size() * sizeof(double2));
    HIPCHK(hipMemcpy(tab.hinv, hi.data(), hi.size() * sizeof(double2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(tab.hmod, hm.data(), hm.size() * sizeof(double2), hipMemcpyHostToDevice));
    tab.pre = tab.post = tab.rinv = nullptr;
    tab.pmod = nullptr;
    if (round) {
        // h = (D - 1)/2 for the (odd) source product D: h mod m = (D mod m - 1) / 2 mod m
        auto half_mod = [&](u64 m) {
            u64 d = 1 % m;
            for (int k = 0; k < tab.ns; k++) d = hmul(d, C.P.mod[src[k]] % m, m);
            return hmul((d + m - 1 % m) % m, hinv(2 % m, m), m);
        };
        std::vector<double> pre(tab.ns), post(tab.nt);
        for (int i = 0; i < tab.ns; i++) pre[i] = (double)half_mod(C.P.mod[src[i]]);
        for (int j = 0; j < tab.nt; j++) post[j] = (double)half_mod(C.P.mod[tgt[j]]);
        tab.pre = (double *)C.table_alloc(pre.size() * sizeof(double));
        tab.post = (double *)C.table_alloc(post.size() * sizeof(double));
        HIPCHK(hipMemcpy(tab.pre, pre.data(), pre.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(tab.post, post.data(), post.size() * sizeof(double), hipMemcpyHostToDevice));
        // exact conversion: 1/p_i for the overflow count, P mod t_j for its removal
        std::vector<double> rinv(tab.ns);
        std::vector<double2> pm(tab.nt);
        for (int i = 0; i < tab.ns; i++) rinv[i] = 1.0 / (double)C.P.mod[src[i]];
        for (int j = 0; j < tab.nt; j++) {
            const u64 t = C.P.mod[tgt[j]];
            u64 d = 1 % t;
            for (int k = 0; k < tab.ns; k++) d = hmul(d, C.P.mod[src[k]] % t, t);
            pm[j] = make_double2((double)d, (double)d / (double)t);
        }
        tab.rinv = (double *)C.table_alloc(rinv.size() * sizeof(double));
        tab.pmod = (double2 *)C.table_alloc(pm.size() * sizeof(double2));
        HIPCHK(hipMemcpy(tab.rinv, rinv.data(), rinv.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(tab.pmod, pm.data(), pm.size() * sizeof(double2), hipMemcpyHostToDevice));
    }
    return tab;
}

// ModUp of digit j at `level`: sources = live primes of the digit, targets =
// every other limb of (q_0..q_level, p_0..p_{K-1}); limb index t in [0, E)
static const BConvTab &modup_tab(Ctx &C, int level, int j) {
    std::lock_guard<std::mutex> g(C.mu);
    auto key = std::make_pair(level, j);
    auto it = C.modup.find(key);
    if (it != C.modup.end()) return it->second;
    const Params &P = C.P;
    const int lo = j * P.alpha, hi = std::min(lo + P.alpha, level + 1) - 1, E = level + 1 + P.K;
    std::vector<int> src, tgt, slot;
    for (int i = lo; i <= hi; i++) src.push_back(i);
    for (int t = 0; t < E; t++) {
        if (t >= lo && t <= hi) continue;
        tgt.push_back(t <= level ? t : P.nq + (t - level - 1));
        slot.push_back(t);
    }
    return C.modup.emplace(key, make_bconv(C, src, tgt, slot)).first->second;
}

static const BConvTab &moddown_tab(Ctx &C, int level) {
    std::lock_guard<std::mutex> g(C.mu);
    auto it = C.moddown.find(level);
    if (it != C.moddown.end()) return it->second;
    std::vector<int> src, tgt, slot;
    for (int k = 0; k < C.P.K; k++) src.push_back(C.P.nq + k);
    for (int i = 0; i <= level; i++) tgt.push_back(i), slot.push_back(i);
    return C.moddown.emplace(level, make_bconv(C, src, tgt, slot, true)).first->second;
}

// ------------------------------------------------------------------------
// evaluator
// ------------------------------------------------------------------------
static void check_same(const DCt &a, const DCt &b) {
    if (a.level != b.level || a.B != b.B) throw Error{CKR_E_INVALID, "level or batch mismatch"};
}

static DCt ev_add(Ctx &C, const DCt &a, const DCt &b, bool sub) {
    check_same(a, b);
    DCt o = ct_new(C, a.level, a.B);
    const size_t L = (size_t)(a.level + 1) * C.n();
    timed(C, kElem, 24.0 * L * a.B * 2, [&] {
        k_add(C.T, o.d(), a.d(), b.d(), a.level + 1, 2 * a.B, L, L, L, plain_map(), sub, C.stream);
    });
    return o;
}

static DCt ev_copy(Ctx &C, const DCt &a) {
    DCt o = ct_new(C, a.level, a.B);
    const size_t words = (size_t)a.B * 2 * (a.level + 1) * C.n();
    timed(C, kCopy, 16.0 * words,
          [&] { HIPCHK(hipMemcpyAsync(o.d(), a.d(), words * 8, hipMemcpyDeviceToDevice, C.stream)); });
    return o;
}

// constant c added to every slot: round(c * D_l) on the constant coefficient
static DCt ev_add_const(Ctx &C, const DCt &a, double c) {
    DCt o = ev_copy(C, a);
    const i64 K = std::llround(c * C.P.scale[a.level]);
    LimbScalars s;
    scalars_of(C, K, a.level + 1, plain_map(), s);
    timed(C, kElem, 16.0 * (a.level + 1) * C.n() * a.B, [&] {
        k_add_scalar(C.T, o.d(), a.level + 1, a.B, (size_t)2 * (a.level + 1) * C.n(), plain_map(), s, C.stream);
    });
    return o;
}

// multiply by a signed integer without rescaling (the scale is unchanged)
static DCt ev_mul_int(Ctx &C, const DCt &a, i64 K) {
    DCt o = ct_new(C, a.level, a.B);
    LimbScalars s;
    scalars_of(C, K, a.level + 1, plain_map(), s);
    const size_t L = (size_t)(a.level + 1) * C.n();
    timed(C, kElem, 16.0 * L * 2 * a.B, [&] {
        k_mul_scalar(C.T, o.d(), a.d(), a.level + 1, 2 * a.B, L, L, plain_map(), s, C.stream);
    });
    return o;
}

// concatenate batches of equal level / split a batch back
static DCt stack(Ctx &C, const std::vector<const DCt *> &parts) {
    int B = 0;
    for (auto *p : parts) {
        if (p->level != parts[0]->level) throw Error{CKR_E_INVALID, "stack: level mismatch"};
        B += p->B;
    }
    DCt o = ct_new(C, parts[0]->level, B);
    const size_t W = (size_t)2 * (o.level + 1) * C.n();
    size_t off = 0;
    for (auto *p : parts) {
        HIPCHK(hipMemcpyAsync(o.d() + off * W, p->d(), p->B * W * 8, hipMemcpyDeviceToDevice, C.stream));
        off += p->B;
    }
    return o;
}
static DCt slice(Ctx &C, const DCt &a, int first, int count) {
    DCt o = ct_new(C, a.level, count);
    const size_t W = (size_t)2 * (a.level + 1) * C.n();
    HIPCHK(hipMemcpyAsync(o.d(), a.d() + first * W, count * W * 8, hipMemcpyDeviceToDevice, C.stream));
    return o;
}

// entries idx[0], idx[1], ... of batch a, in that order
static DCt gather(Ctx &C, const DCt &a, const std::vector<int> &idx) {
    DCt o = ct_new(C, a.level, (int)idx.size());
    const size_t W = (size_t)2 * (a.level + 1) * C.n();
    for (size_t k = 0; k < idx.size(); k++)
        HIPCHK(hipMemcpyAsync(o.d() + k * W, a.d() + (size_t)idx[k] * W, W * 8, hipMemcpyDeviceToDevice, C.stream));
    return o;
}

// rounding rescale: c_i <- (c_i - [v]_{q_i}) * q_l^{-1} mod q_i, v the last
// limb's residue taken in (-q_l/2, q_l/2), i.e. floor((X + (q_l - 1)/2) / q_l)
// (a floor would leave every coefficient about 1/2 low: a constant bias that
// slot 0 amplifies the most).  The last limb is brought to the coefficient
// domain, then one fused forward transform reduces it modulo every q_i
// (prologue) and writes the combined result (epilogue).
static DCt ev_rescale(Ctx &C, const DCt &a) {
    const int l = a.level;
    if (l < 1) throw Error{CKR_E_DEPTH, "rescale at level 0"};
    const size_t n = C.n(), L = (size_t)(l + 1) * n;
    const int P2 = 2 * a.B;
    Buf last(&C, (size_t)P2 * n);
    ntt(C, last.get(), 1, P2, n, plain_map(l), true, a.d() + (size_t)l * n, L);
    DCt o = ct_new(C, l - 1, a.B);
    std::vector<u64> inv(l);
    for (int i = 0; i < l; i++) inv[i] = hinv(C.P.mod[l] % C.P.mod[i], C.P.mod[i]);
    NttFuse f;
    f.pro = true;
    f.pro_q = (double)C.P.mod[l];
    f.src = last.get();
    f.src_stride = n;
    f.epi = true;
    f.out = o.d();
    f.out_stride = (size_t)2 * l * n;
    f.out_off = (size_t)l * n;
    f.x = a.d();
    f.x_stride = 2 * L;
    f.x_off = L;
    scalars_of_vals(C, inv, f.c);
    Buf y(&C, (size_t)P2 * l * n);
    ntt_fused(C, y.get(), l, P2, (size_t)l * n, plain_map(), f);
    return o;
}

// c * a brought to level `target`: drop to target+1 limbs, multiply by
// round(c * D_target * q_{target+1} / D_level), rescale by q_{target+1}
// The product by K rides in the rescale: limb l2 of K a is formed alone and
// brought to the coefficient domain, and the rescale's fused transform of
// limbs 0..l2-1 takes (x K - y) q_{l2}^{-1} in its epilogue, the same residues
// as rescaling the full product.
static DCt ev_cmul_to(Ctx &C, const DCt &a, double c, int target, const DCt *plus = nullptr, bool minus = false) {
    if (target < 0 || target >= a.level) throw Error{CKR_E_DEPTH, "cmul_to target"};
    if (plus && (plus->level != target || plus->B != a.B)) throw Error{CKR_E_INVALID, "cmul_to addend"};
    const double v = ((c * C.P.scale[target]) * (double)C.P.mod[target + 1]) / C.P.scale[a.level];
    const i64 K = std::llround(v);
    const int l2 = target + 1;
    const size_t n = C.n(), La = (size_t)(a.level + 1) * n;
    const int P2 = 2 * a.B;
    // K times limb l2, then its coefficients
    Buf ml(&C, (size_t)P2 * n);
    LimbScalars sl;
    scalars_of(C, K, 1, plain_map(l2), sl);
    timed(C, kElem, 16.0 * n * P2, [&] {
        k_mul_scalar(C.T, ml.get(), a.d() + (size_t)l2 * n, 1, P2, n, La, plain_map(l2), sl, C.stream);
    });
    Buf last(&C, (size_t)P2 * n);
    ntt(C, last.get(), 1, P2, n, plain_map(l2), true, ml.get(), n);
    DCt o = ct_new(C, target, a.B);
    std::vector<u64> inv(l2);
    for (int i = 0; i < l2; i++) inv[i] = hinv(C.P.mod[l2] % C.P.mod[i], C.P.mod[i]);
    NttFuse f;
    f.pro = true;
    f.pro_q = (double)C.P.mod[l2];
    f.src = last.get();
    f.src_stride = n;
    f.epi = true;
    f.pre = true;
    f.out = o.d();
    f.out_stride = (size_t)2 * l2 * n;
    f.out_off = (size_t)l2 * n;
    f.x = a.d();
    f.x_stride = 2 * La;
    f.x_off = La;
    if (plus) {  // + plus (- plus when minus), after the rescale
        f.add2 = plus->d();
        f.add2_stride = (size_t)2 * l2 * n;
        f.add2_off = (size_t)l2 * n;
        f.add2_mask = 3;
        f.add2_sub = minus;
    }
    scalars_of_vals(C, inv, f.c);
    scalars_of(C, K, l2, plain_map(), f.c2);
    Buf y(&C, (size_t)P2 * l2 * n);
    ntt_fused(C, y.get(), l2, P2, (size_t)l2 * n, plain_map(), f);
    return o;
}

// The relinearisation's ModDown and the rescale after it, in one pass over
// limbs 0..l-1 (multiplication's tail).  With x the key inner product (eval
// domain), b = conv the ModDown base conversion (coefficient domain) and d the
// tensor's (d0, d1), the switched ciphertext is r = (x - NTT(b)) P^{-1} + d,
// and the rescale gives o_i = (r_i - NTT([v]_{q_i})) q_l^{-1}, v = INTT(r_l)
// taken in (-q_l/2, q_l/2).  NTT is linear, so
//   o_i = (x_i P^{-1} + d_i - NTT(b_i P^{-1} + [v]_{q_i})) q_l^{-1}:
// limb l of r is formed first (the ModDown epilogue on that limb alone) and
// brought to the coefficient domain; then one fused forward transform of
// limbs 0..l-1 adds [v]_{q_i} and b_i P^{-1} in its prologue and combines in
// its epilogue.  Every operation is modular, so o is the same residues as the
// ModDown followed by the rescale, and the switched ciphertext at level l
// never reaches HBM.
static void moddown_rescale(Ctx &C, u64 *conv, const u64 *acc, size_t sacc, int E, int l, int B,
                            const std::vector<u64> &pinv, const u64 *d, size_t sd, size_t d_off, DCt &o) {
    const size_t n = C.n();
    const int P2 = 2 * B;
    // r_l = (x_l - NTT(b_l)) P^{-1} + d_l, then its coefficients
    Buf rl(&C, (size_t)P2 * n);
    NttFuse f1;
    f1.epi = true;
    f1.out = rl.get();
    f1.out_stride = 2 * n;
    f1.out_off = n;
    f1.x = acc + (size_t)l * n;
    f1.x_stride = sacc;
    f1.x_off = (size_t)E * n;
    f1.add = d + (size_t)l * n;
    f1.add_stride = sd;
    f1.add_off = d_off;
    f1.add_mask = 3;
    f1.c.v[0] = (double)pinv[l];  // limb 0 of this one-limb transform is modulus l
    f1.c.vq[0] = (double)pinv[l] / (double)C.P.mod[l];
    ntt_fused(C, conv + (size_t)l * n, 1, P2, (size_t)(l + 1) * n, plain_map(l), f1);
    Buf last(&C, (size_t)P2 * n);
    ntt(C, last.get(), 1, P2, n, plain_map(l), true, rl.get(), n);
    // limbs 0..l-1
    std::vector<u64> qlinv(l), pv(pinv.begin(), pinv.begin() + l);
    for (int i = 0; i < l; i++) qlinv[i] = hinv(C.P.mod[l] % C.P.mod[i], C.P.mod[i]);
    NttFuse f;
    f.pro = true;
    f.pro_q = (double)C.P.mod[l];
    f.src = last.get();
    f.src_stride = n;
    f.src2 = conv;
    f.src2_stride = (size_t)(l + 1) * n;
    f.epi = true;
    f.pre = true;
    f.out = o.d();
    f.out_stride = (size_t)2 * l * n;
    f.out_off = (size_t)l * n;
    f.x = acc;
    f.x_stride = sacc;
    f.x_off = (size_t)E * n;
    f.add = d;
    f.add_stride = sd;
    f.add_off = d_off;
    f.add_mask = 3;
    scalars_of_vals(C, qlinv, f.c);
    scalars_of_vals(C, pv, f.c2);
    Buf y(&C, (size_t)P2 * l * n);
    ntt_fused(C, y.get(), l, P2, (size_t)l * n, plain_map(), f);
}

// hybrid key switch of d (B polys, eval domain, limbs 0..l, batch stride sd):
//   out_b = ModDown(sum_j ModUp_j(d) * key_j.b) (+ add_b),  out_a likewise
// Output poly k (0: b part, 1: a part) of batch entry b goes to out + b*so + k*out_off
// and, when bit k of add_mask is set, has add + b*sadd + k*add_off added.
// With gal > 1, d and add are read through the automorphism sigma_gal: the
// rotation's permutation rides in the key switch's loads.
static void keyswitch(Ctx &C, const Keys &K, const Buf &key, const u64 *d, size_t sd, int l, int B, u64 *out,
                      size_t so, size_t out_off, const u64 *add, size_t sadd, size_t add_off, int add_mask,
                      const u64 *add2 = nullptr, size_t sadd2 = 0, size_t add2_off = 0, int add2_mask = 0,
                      u32 gal = 0, DCt *rescaled = nullptr) {
    const Params &P = C.P;
    if (l > K.lmax) throw Error{CKR_E_DEPTH, "ciphertext above key level"};
    const size_t n = C.n();
    const int beta = P.beta(l), E = l + 1 + P.K;
    // coefficient-domain copy of d
    Buf dc(&C, (size_t)B * (l + 1) * n);
    ntt(C, dc.get(), l + 1, B, (size_t)(l + 1) * n, plain_map(), true, d, sd, gal);
    // ModUp: base conversion of each digit to the other limbs, then NTT
    const size_t sext = (size_t)beta * E * n;
    Buf ext(&C, (size_t)B * sext);
    for (int j = 0; j < beta; j++) {
        const int lo = j * P.alpha, hi = std::min(lo + P.alpha, l + 1) - 1;
        u64 *ej = ext.get() + (size_t)j * E * n;
        const BConvTab &tab = modup_tab(C, l, j);
        timed(C, kBConv, 8.0 * n * (tab.ns + tab.nt) * B, [&] {
            k_bconv(C.T, ej, dc.get() + (size_t)lo * n, tab, B, sext, (size_t)(l + 1) * n, C.stream);
        });
        // column pass only: the row pass runs fused with the inner product below
        if (lo > 0) ntt_first(C, ej, lo, B, sext, plain_map());
        if (hi + 1 < E) ntt_first(C, ej + (size_t)(hi + 1) * n, E - hi - 1, B, sext, LimbMap{l - hi, hi + 1, P.nq});
    }
    // row pass + inner product with the key digits
    const size_t sacc = (size_t)2 * E * n;
    Buf acc(&C, (size_t)B * sacc);
    IPArgs ia;
    ia.d = d;
    ia.ext = ext.get();
    ia.key = key.get();
    ia.accb = acc.get();
    ia.acca = acc.get() + (size_t)E * n;
    ia.level = l;
    ia.E = E;
    ia.beta = beta;
    ia.alpha = P.alpha;
    ia.Ek = K.Ek();
    ia.lmax_key = K.lmax;
    ia.nq = P.nq;
    ia.B = B;
    ia.sd = sd;
    ia.sext = sext;
    ia.sacc = sacc;
    ia.gal = gal;
    ia.inv_p = true;  // the special-prime limbs leave after ModDown's first inverse pass
    // per target limb: beta inputs and 2 outputs per batch entry, 2*beta key limbs once
    timed(C, kNttRowIP, 8.0 * n * E * ((beta + 2.0) * B + 2.0 * beta), [&] { k_ntt_row_ip(C.T, ia, C.stream); });
    // ModDown, rounding: (x_Q + h - [(X + h) mod P]_Q) * P^{-1} = round(X / P), h = (P - 1)/2
    // (both h's folded into the exact base conversion), the combine fused into the last NTT pass.
    // The inverse transform of the special-prime limbs: its row pass ran in the kernel above.
    intt_second(C, acc.get() + (size_t)(l + 1) * n, P.K, 2 * B, (size_t)E * n, plain_map(P.nq));
    Buf conv(&C, (size_t)2 * B * (l + 1) * n);
    const BConvTab &mdt = moddown_tab(C, l);
    timed(C, kBConv, 8.0 * n * (mdt.ns + mdt.nt) * 2 * B, [&] {
        k_bconv(C.T, conv.get(), acc.get() + (size_t)(l + 1) * n, mdt, 2 * B, (size_t)(l + 1) * n, (size_t)E * n,
                C.stream);
    });
    std::vector<u64> pinv(l + 1);
    for (int i = 0; i <= l; i++) {
        const u64 q = P.mod[i];
        u64 pp = 1 % q;
        for (int k = 0; k < P.K; k++) pp = hmul(pp, P.mod[P.nq + k] % q, q);
        pinv[i] = hinv(pp, q);
    }
    if (rescaled) {
        moddown_rescale(C, conv.get(), acc.get(), sacc, E, l, B, pinv, add, sadd, add_off, *rescaled);
        return;
    }
    NttFuse f;
    f.epi = true;
    f.out = out;
    f.out_stride = so;
    f.out_off = out_off;
    f.x = acc.get();
    f.x_stride = sacc;
    f.x_off = (size_t)E * n;
    f.add = add;
    f.add_stride = sadd;
    f.add_off = add_off;
    f.add_mask = add ? add_mask : 0;
    f.add_gal = gal;
    f.add2 = add2;
    f.add2_stride = sadd2;
    f.add2_off = add2_off;
    f.add2_mask = add2 ? add2_mask : 0;
    scalars_of_vals(C, pinv, f.c);
    ntt_fused(C, conv.get(), l + 1, 2 * B, (size_t)(l + 1) * n, plain_map(), f);
}

static const Buf &find_key(const Keys &K, u32 g) {
    auto it = K.swk.find(g);
    if (it == K.swk.end()) throw Error{CKR_E_INVALID, "missing switching key for galois element " + std::to_string(g)};
    return it->second;
}

// ct * ct: tensor, relinearise with the s^2 key, rescale
static DCt ev_mul(Ctx &C, const Keys &K, const DCt &a, const DCt &b) {
    check_same(a, b);
    const int l = a.level;
    if (l < 1) throw Error{CKR_E_DEPTH, "mul at level 0"};
    const size_t n = C.n(), L = (size_t)(l + 1) * n;
    Buf d(&C, (size_t)a.B * 3 * L);
    timed(C, kTensor, 56.0 * L * a.B, [&] { k_tensor(C.T, d.get(), a.d(), b.d(), l + 1, a.B, 3 * L, 2 * L, 2 * L, C.stream); });
    // (d0 + KS_b(d2), d1 + KS_a(d2)) rescaled, the ModDown and the rescale in one pass
    DCt o = ct_new(C, l - 1, a.B);
    keyswitch(C, K, find_key(K, 0), d.get() + 2 * L, 3 * L, l, a.B, nullptr, 0, 0, d.get(), 3 * L, L, 3, nullptr, 0,
              0, 0, 0, &o);
    return o;
}

static u32 galois_left(const Ctx &C, i64 k) {
    const i64 h = (i64)(C.n() / 2);
    const u64 kk = (u64)(((k % h) + h) % h);
    return (u32)hpow(5, kk, 2 * C.n());
}

// left rotation by k (new[j] = old[j+k]); k < 0 rotates right
static DCt ev_rotate(Ctx &C, const Keys &K, const DCt &a, i64 k) {
    const u32 g = galois_left(C, k);
    if (g == 1) return ev_copy(C, a);
    const Buf &key = find_key(K, g);
    const int l = a.level;
    const size_t n = C.n(), L = (size_t)(l + 1) * n;
    DCt o = ct_new(C, l, a.B);
    // (sigma(c0) + KS_b(sigma(c1)), KS_a(sigma(c1))), sigma applied while reading c0 and c1
    keyswitch(C, K, key, a.d() + L, 2 * L, l, a.B, o.d(), 2 * L, L, a.d(), 2 * L, L, 1, nullptr, 0, 0, 0, g);
    return o;
}

// X + sigma_g(X): the addition rides in the key switch's epilogue
static DCt ev_galois_add(Ctx &C, const Keys &K, const DCt &a, u32 g) {
    if (g == 1) return ev_add(C, a, a, false);
    const Buf &key = find_key(K, g);
    const int l = a.level;
    const size_t n = C.n(), L = (size_t)(l + 1) * n;
    DCt o = ct_new(C, l, a.B);
    // (a0 + sigma(a0) + KS_b(sigma(a1)), a1 + KS_a(sigma(a1))), sigma applied while reading a0 and a1
    keyswitch(C, K, key, a.d() + L, 2 * L, l, a.B, o.d(), 2 * L, L, a.d(), 2 * L, L, 1, a.d(), 2 * L, L, 3, g);
    return o;
}

// X + (X rotated left by k)
static DCt ev_rotate_add(Ctx &C, const Keys &K, const DCt &a, i64 k) { return ev_galois_add(C, K, a, galois_left(C, k)); }

// A Chebyshev indicator of degree 2^(D-1) - 1 grows like cosh(n y / sqrt(1 - x^2))
// at x + iy, and its argument inherits imaginary parts (the comparator's
// slope amplifies the slots' imaginary noise): the argument is projected onto
// its real part as X + conj(X), conj = sigma_{2n-1}, with the factor 1/2
// folded into the scaling before it.
static DCt ev_plus_conj(Ctx &C, const Keys &K, const DCt &a) { return ev_galois_add(C, K, a, (u32)(2 * C.n() - 1)); }

// plaintext holding z on slots [0, count) at scale D_level, eval domain [level+1][n]
enum PlainKind { kMaskRow0 = 1, kMaskCol0 = 2, kHalfRow0 = 3, kTieMask = 4, kSteps = 5, kNegHalfRow0 = 6,
                 kStepsBlock = 7, kHalfCol0 = 8, kStepsCol = 9, kBlockMask = 10 };

static Buf encode_plain(Ctx &C, const std::vector<double> &z, int level) {
    const size_t n = C.n();
    std::vector<i64> m(n);
    if (!encode_slots(C.P.logn, z.data(), (u32)z.size(), C.P.scale[level], m.data()))
        throw Error{CKR_E_RANGE, "plaintext coefficient overflow"};
    std::vector<u64> res((size_t)(level + 1) * n);
    for (int t = 0; t <= level; t++)
        for (size_t j = 0; j < n; j++) res[(size_t)t * n + j] = hred(m[j], C.P.mod[t]);
    Buf b(&C, res.size());
    HIPCHK(hipMemcpyAsync(b.get(), res.data(), res.size() * 8, hipMemcpyHostToDevice, C.stream));
    ntt(C, b.get(), level + 1, 1, (size_t)(level + 1) * n, plain_map(), false);
    sync(C);  // res goes out of scope
    return b;
}

static std::vector<double> plain_values(int kind, int N, int arg) {
    std::vector<double> z((size_t)N * N, 0.0);
    switch (kind) {
    case kMaskRow0: for (int j = 0; j < N; j++) z[j] = 1.0; break;
    case kMaskCol0: for (int i = 0; i < N; i++) z[(size_t)i * N] = 1.0; break;
    case kHalfRow0: z.assign(N, 0.5); break;
    case kNegHalfRow0: z.assign(N, -0.5); break;
    case kTieMask:  // delta_{j >= i} - 1/2 on the N x N block
        for (int i = 0; i < N; i++)
            for (int j = 0; j < N; j++) z[(size_t)i * N + j] = (j >= i) ? 0.5 : -0.5;
        break;
    case kSteps:  // -(1^N || 2^N || ... || N^N)
        for (int i = 0; i < N; i++)
            for (int j = 0; j < N; j++) z[(size_t)i * N + j] = -(double)(i + 1);
        break;
    case kStepsBlock:  // -((N arg + 1)^N || ... || (N arg + N)^N): the ranks of output block arg
        for (int i = 0; i < N; i++)
            for (int j = 0; j < N; j++) z[(size_t)i * N + j] = -((double)N * arg + i + 1);
        break;
    case kBlockMask:  // 1 on the arg x arg block of the N x N layout
        for (int i = 0; i < arg; i++)
            for (int j = 0; j < arg; j++) z[(size_t)i * N + j] = 1.0;
        break;
    case kHalfCol0:  // 1/2 on column 0
        for (int i = 0; i < N; i++) z[(size_t)i * N] = 0.5;
        break;
    case kStepsCol:  // -(1 || 2 || ... || N)^N: column k holds -(k + 1)
        for (int i = 0; i < N; i++)
            for (int j = 0; j < N; j++) z[(size_t)i * N + j] = -(double)(j + 1);
        break;
    default: throw Error{CKR_E_INVALID, "plaintext kind"};
    }
    return z;
}

static const Buf &get_plain(Ctx &C, int kind, int N, int level, int arg = 0) {
    PlainKey key{kind, N, level, arg};
    {
        std::lock_guard<std::mutex> g(C.mu);
        auto it = C.plain.find(key);
        if (it != C.plain.end()) return it->second;
    }
    Buf b = encode_plain(C, plain_values(kind, N, arg), level);
    std::lock_guard<std::mutex> g(C.mu);
    return C.plain.emplace(key, std::move(b)).first->second;
}

// slot-wise product with a plaintext (eval domain), then rescale.  As for a
// constant product, only the dropped limb's product is formed ahead (and
// brought to the coefficient domain); the rescale's fused transform takes
// (x pt - y) q_l^{-1} in its epilogue: the same residues as rescaling the
// full product, which is never written.
static DCt ev_mul_plain(Ctx &C, const DCt &a, const Buf &pt) {
    const int l = a.level;
    if (l < 1) throw Error{CKR_E_DEPTH, "rescale at level 0"};
    const size_t n = C.n(), L = (size_t)(l + 1) * n;
    const int P2 = 2 * a.B;
    Buf ml(&C, (size_t)P2 * n);
    timed(C, kElem, 8.0 * n * (4 * a.B + 1), [&] {
        k_mul_pt(C.T, ml.get(), a.d() + (size_t)l * n, pt.get() + (size_t)l * n, 1, P2, n, L, plain_map(l), false,
                 C.stream);
    });
    Buf last(&C, (size_t)P2 * n);
    ntt(C, last.get(), 1, P2, n, plain_map(l), true, ml.get(), n);
    DCt o = ct_new(C, l - 1, a.B);
    std::vector<u64> inv(l);
    for (int i = 0; i < l; i++) inv[i] = hinv(C.P.mod[l] % C.P.mod[i], C.P.mod[i]);
    NttFuse f;
    f.pro = true;
    f.pro_q = (double)C.P.mod[l];
    f.src = last.get();
    f.src_stride = n;
    f.epi = true;
    f.xmul = pt.get();
    f.out = o.d();
    f.out_stride = (size_t)2 * l * n;
    f.out_off = (size_t)l * n;
    f.x = a.d();
    f.x_stride = 2 * L;
    f.x_off = L;
    scalars_of_vals(C, inv, f.c);
    Buf y(&C, (size_t)P2 * l * n);
    ntt_fused(C, y.get(), l, P2, (size_t)l * n, plain_map(), f);
    return o;
}

static DCt ev_add_plain(Ctx &C, const DCt &a, const Buf &pt) {
    const size_t L = (size_t)(a.level + 1) * C.n();
    DCt o = ev_copy(C, a);
    timed(C, kElem, 8.0 * L * (2 * a.B + 1), [&] {
        k_mul_pt(C.T, o.d(), a.d(), pt.get(), a.level + 1, a.B, 2 * L, 2 * L, plain_map(), true, C.stream);
    });
    return o;
}

// ------------------------------------------------------------------------
// matrix operations (section 2.3, Algorithms TransR/TransC, Appendix A)
// ------------------------------------------------------------------------
static int lg(int N) {
    int r = 0;
    while ((1 << r) < N) r++;
    return r;
}

// X_{i+1} = X_i + rot(X_i, shift(i)) for i in [from, to), starting from V
template <class Shift>
static DCt rot_add_chain(Ctx &C, const Keys &K, const DCt &V, int from, int to, Shift shift) {
    DCt X;
    const DCt *cur = &V;
    for (int i = from; i < to; i++) {
        X = ev_rotate_add(C, K, *cur, shift(i));
        cur = &X;
    }
    return cur == &V ? ev_copy(C, V) : std::move(X);
}

static DCt trans_r(Ctx &C, const Keys &K, const DCt &V, int N) {
    DCt X = rot_add_chain(C, K, V, 1, lg(N) + 1, [&](int i) { return -(i64)(((i64)N * (N - 1)) >> i); });
    return ev_mul_plain(C, X, get_plain(C, kMaskCol0, N, X.level));
}
static DCt trans_c(Ctx &C, const Keys &K, const DCt &V, int N) {
    DCt X = rot_add_chain(C, K, V, 1, lg(N) + 1, [&](int i) { return (i64)(((i64)N * (N - 1)) >> i); });
    return ev_mul_plain(C, X, get_plain(C, kMaskRow0, N, X.level));
}
static DCt sum_r(Ctx &C, const Keys &K, const DCt &V, int N) {
    DCt X = rot_add_chain(C, K, V, 0, lg(N), [&](int i) { return (i64)N << i; });
    return ev_mul_plain(C, X, get_plain(C, kMaskRow0, N, X.level));
}
static DCt sum_c(Ctx &C, const Keys &K, const DCt &V, int N) {
    DCt X = rot_add_chain(C, K, V, 0, lg(N), [&](int i) { return (i64)1 << i; });
    return ev_mul_plain(C, X, get_plain(C, kMaskCol0, N, X.level));
}
static DCt repl_r(Ctx &C, const Keys &K, const DCt &V, int N) {
    return rot_add_chain(C, K, V, 0, lg(N), [&](int i) { return -((i64)N << i); });
}
static DCt repl_c(Ctx &C, const Keys &K, const DCt &V, int N) {
    return rot_add_chain(C, K, V, 0, lg(N), [&](int i) { return -((i64)1 << i); });
}

// ------------------------------------------------------------------------
// comparator: f/g composite of odd degree-7 polynomials (section 2.2)
// ------------------------------------------------------------------------
static const double kF[4] = {35.0 / 16, -35.0 / 16, 21.0 / 16, -5.0 / 16};
static const double kG[4] = {4589.0 / 1024, -16577.0 / 1024, 25614.0 / 1024, -12860.0 / 1024};
// Minimax composite (section 2.2's alternative to f and g: composite minimax
// approximations of the sign function): stage 0 is the odd degree-7
// polynomial closest to 1 in the maximum norm on [2^-8.5, 1], stage s the one
// closest to 1 on the interval stage s-1 maps that onto (errors 0.968, 0.827,
// 0.362, 9.8e-3, 5.1e-9).  Coefficients of x, x^3, x^5, x^7.
constexpr int kMinimaxStages = 5;
static const double kMM[kMinimaxStages][4] = {
    {11.626630381861787, -68.36534054680979, 126.44790262989271, -69.67707957286088},
    {5.38484717173034, -7.907363201737443, 3.7393070660732937, -0.5295271268765817},
    {3.8547436306459173, -5.358791130620638, 2.7473565274453287, -0.4363096838044091},
    {2.363269725894833, -2.5537068630909263, 1.5095093062451124, -0.32798232661912397},
    {2.1876161909909757, -2.187742945230383, 1.3126373118789916, -0.3125105627390891},
};

// a1 x + a3 x^3 + a5 x^5 + a7 x^7 (a7 != 0) in three levels and four products:
//   y = x^2, t = (a7 x) y = a7 x^3, y2 = y^2, h = y2 (t + a5 x) = a7 x^7 + a5 x^5,
//   result = h + (a3/a7) t + a1 x, the last two brought down to level l-3 by
//   constant products (a3 x^3 from t instead of a fifth ciphertext product)
static DCt poly7(Ctx &C, const Keys &K, const DCt &x, const double a[4]) {
    const int l = x.level;
    if (l < 3) throw Error{CKR_E_DEPTH, "poly7 needs three levels"};
    if (a[3] == 0.0) throw Error{CKR_E_INVALID, "poly7 needs a degree-7 term"};
    // x^2 runs beside a7 x, then y^2 beside (a7 x) y: two branches each
    DCt y, c3, t, y2;
    {
        Branches br(C);
        br.run([&] { c3 = ev_cmul_to(C, x, a[3], l - 1); });
        y = ev_mul(C, K, x, x);
        br.join();
    }
    {
        Branches br(C);
        br.run([&] { y2 = ev_mul(C, K, y, y); });
        t = ev_mul(C, K, c3, y);
        br.join();
    }
    DCt w = ev_cmul_to(C, x, a[2], l - 2, &t);              // t + a5 x
    DCt h = ev_mul(C, K, y2, w);
    DCt s1 = ev_cmul_to(C, t, a[1] / a[3], l - 3, &h);      // h + (a3/a7) t
    return ev_cmul_to(C, x, a[0], l - 3, &s1);              // + a1 x
}

// ------------------------------------------------------------------------
// Chebyshev comparator (section 2.2): the comparison function as a function
// of d = x - y, interpolated at the 2^(D-1) Chebyshev nodes of [-1, 1] and
// evaluated by the Paterson-Stockmeyer algorithm in the Chebyshev basis.
// For sum_{i < 2^B} c_i T_i(x): k = 2^l baby steps (l = ceil(B/2)) and
// m = B - l giant steps,
//   T_1 = x, T_{2j} = 2 T_j^2 - 1, T_{2j+1} = 2 T_j T_{j+1} - T_1,
//   G_0 = T_k, G_r = 2 G_{r-1}^2 - 1,
// and p = q G_{r-1} + s recursively (Chebyshev division by T_K, K = k 2^(r-1):
// q_0 = c_K, q_j = 2 c_{K+j}, s_0 = c_0, s_i = c_i - c_{2K-i}) down to
// polynomials of degree < k, each a linear combination of the baby steps
// brought to one level (integer constants, one rescale, then + c_0).  x at
// level L leaves at level L - B - 1.
//
// On the GPU every stage runs batched: the baby steps of one level form one
// product batch, all 2^m linear combinations are one fused kernel over the
// baby steps, and each level of the division tree is one product batch.
// The leaves are ordered so that the tree folds by halves: leaf index =
// sum_r choice_r 2^(m-r), choice_r = 0 for the quotient, 1 for the
// remainder of the split at tree level r (r = m at the root).
// ------------------------------------------------------------------------
constexpr int kChebMaxDepth = 16;
constexpr int kChebChunk = 256;  // batch entries per product launch in the Chebyshev evaluation

static int cmp_levels(ckr_sign c) { return c.cheb ? c.cheb : 3 * (c.d_g + c.d_f + c.minimax); }

static void cheb_split(const std::vector<double> &c, int k, int r, int m, int idx,
                       std::vector<std::vector<double>> &leaves) {
    if (r == 0) {
        leaves[idx] = c;
        return;
    }
    const int K = k << (r - 1);
    std::vector<double> q(K), s(K);
    q[0] = c[K];
    s[0] = c[0];
    for (int j = 1; j < K; j++) {
        q[j] = 2.0 * c[K + j];
        s[j] = c[j] - c[2 * K - j];
    }
    cheb_split(q, k, r - 1, m, idx, leaves);
    cheb_split(s, k, r - 1, m, idx + (1 << (m - r)), leaves);
}

// per-limb constants of the linear combinations: [leaf][term][limb] at level lb
static const Buf &lincomb_table(Ctx &C, const std::vector<std::vector<double>> &leaves, const std::vector<int> &terms,
                                int lb) {
    std::vector<u64> key;
    key.push_back((u64)lb);
    for (int i : terms) key.push_back((u64)i);
    for (const auto &lf : leaves)
        for (int i : terms) {
            u64 b;
            std::memcpy(&b, &lf[i], 8);
            key.push_back(b);
        }
    {
        std::lock_guard<std::mutex> g(C.mu);
        auto it = C.lincomb.find(key);
        if (it != C.lincomb.end()) return it->second;
    }
    const int t = lb - 1, limbs = lb + 1;
    std::vector<double2> tab(leaves.size() * terms.size() * limbs);
    size_t w = 0;
    for (const auto &lf : leaves)
        for (int i : terms) {
            const i64 K = std::llround(((lf[i] * C.P.scale[t]) * (double)C.P.mod[t + 1]) / C.P.scale[lb]);
            for (int l = 0; l < limbs; l++) {
                const u64 q = C.P.mod[l], v = hred(K, q);
                tab[w++] = double2{(double)v, (double)v / (double)q};
            }
        }
    Buf b(&C, tab.size() * 2);
    HIPCHK(hipMemcpyAsync(b.get(), tab.data(), tab.size() * sizeof(double2), hipMemcpyHostToDevice, C.stream));
    sync(C);  // tab goes out of scope
    std::lock_guard<std::mutex> g(C.mu);
    return C.lincomb.emplace(std::move(key), std::move(b)).first->second;
}

// x brought to `level` (none of the work when it is already there)
static const DCt &aligned(Ctx &C, const DCt &x, int level, DCt &store) {
    if (x.level == level) return x;
    store = ev_cmul_to(C, x, 1.0, level);
    return store;
}

// pairs (a_i, b_i) multiplied, doubled and reduced by s_i (nullptr: by 1),
// in product launches of at most kChebChunk entries; every a_i, b_i at one level
static std::vector<DCt> cheb_steps(Ctx &C, const Keys &K, const std::vector<const DCt *> &a,
                                   const std::vector<const DCt *> &b, const DCt *s) {
    std::vector<DCt> out;
    const int B = a[0]->B;
    const int per = std::max(1, kChebChunk / B);
    for (size_t c0 = 0; c0 < a.size(); c0 += per) {
        const size_t c1 = std::min(a.size(), c0 + per);
        std::vector<const DCt *> la(a.begin() + c0, a.begin() + c1), lb(b.begin() + c0, b.begin() + c1);
        DCt P = ev_mul_int(C, ev_mul(C, K, stack(C, la), stack(C, lb)), 2);
        DCt sub;
        if (s) {
            DCt sa;
            const DCt &S = aligned(C, *s, P.level, sa);
            std::vector<const DCt *> rep(c1 - c0, &S);
            sub = ev_add(C, P, stack(C, rep), true);
        } else {
            sub = ev_add_const(C, P, -1.0);
        }
        for (size_t i = 0; i < c1 - c0; i++) out.push_back(slice(C, sub, (int)i * B, B));
    }
    return out;
}

static DCt cheb_eval(Ctx &C, const Keys &K, const DCt &x, const std::vector<double> &c) {
    const int deg1 = (int)c.size();
    int Bd = 0;
    while ((1 << Bd) < deg1) Bd++;
    if (deg1 < 2 || (1 << Bd) != deg1 || Bd + 1 > kChebMaxDepth)
        throw Error{CKR_E_INVALID, "Chebyshev series length must be a power of two in [2, 2^15]"};
    if (x.level < Bd + 1) throw Error{CKR_E_DEPTH, "not enough levels for the Chebyshev series"};
    const int l = (Bd + 1) / 2, m = Bd - l, k = 1 << l, top = m > 0 ? k : k - 1, B = x.B;
    const int lb = x.level - l;

    // division tree and the baby steps its leaves use (T_1 always)
    std::vector<std::vector<double>> leaves((size_t)1 << m);
    cheb_split(c, k, m, m, 0, leaves);
    std::vector<int> terms{1};
    for (int i = 2; i < k; i++)
        for (const auto &lf : leaves)
            if (lf[i] != 0.0) {
                terms.push_back(i);
                break;
            }
    if ((int)terms.size() > kMaxLinTerms) throw Error{CKR_E_INVALID, "too many baby steps"};

    // baby steps by level: T_j for j in (2^(r-1), 2^r] from operands at level x.level - (r-1)
    std::vector<DCt> T(top + 1);
    std::vector<const DCt *> Tp(top + 1, nullptr);
    Tp[1] = &x;
    for (int r = 1; r <= l; r++) {
        const int lo = std::max(2, (1 << (r - 1)) + 1), hi = std::min(1 << r, top);
        if (lo > hi) continue;
        const int lev = x.level - (r - 1);
        std::map<int, DCt> al;
        auto op = [&](int i) -> const DCt * {
            if (Tp[i]->level == lev) return Tp[i];
            auto it = al.find(i);
            if (it == al.end()) it = al.emplace(i, ev_cmul_to(C, *Tp[i], 1.0, lev)).first;
            return &it->second;
        };
        std::vector<int> odd, even;
        for (int j = lo; j <= hi; j++) (j & 1 ? odd : even).push_back(j);
        for (int pass = 0; pass < 2; pass++) {
            const std::vector<int> &js = pass == 0 ? odd : even;
            if (js.empty()) continue;
            std::vector<const DCt *> a, b;
            for (int j : js) {
                a.push_back(op(j / 2));
                b.push_back(op(pass == 0 ? j / 2 + 1 : j / 2));
            }
            std::vector<DCt> res = cheb_steps(C, K, a, b, pass == 0 ? &x : nullptr);
            for (size_t i = 0; i < js.size(); i++) {
                T[js[i]] = std::move(res[i]);
                Tp[js[i]] = &T[js[i]];
            }
        }
    }

    // the used baby steps at level lb, then every leaf combination in one kernel
    std::vector<DCt> Tb(k);
    LinComb lc{};
    lc.nt = (int)terms.size();
    lc.nout = (int)leaves.size();
    lc.limbs = lb + 1;
    lc.B = B;
    for (int i = 0; i < lc.nt; i++) {
        const int ti = terms[i];
        const DCt &src = aligned(C, *Tp[ti], lb, Tb[ti]);
        lc.term[i] = src.d();
    }
    DCt Y = ct_new(C, lb, lc.nout * B);
    lc.out = Y.d();
    lc.k = (const double2 *)lincomb_table(C, leaves, terms, lb).get();
    timed(C, kElem, 8.0 * (lc.nt + lc.nout) * 2.0 * lc.limbs * C.n() * B, [&] { k_lincomb(C.T, lc, C.stream); });
    Y = ev_rescale(C, Y);
    const size_t W = (size_t)2 * (Y.level + 1) * C.n();
    for (int j = 0; j < lc.nout; j++) {
        LimbScalars cs;
        scalars_of(C, std::llround(leaves[j][0] * C.P.scale[Y.level]), Y.level + 1, plain_map(), cs);
        timed(C, kElem, 16.0 * (Y.level + 1) * C.n() * B, [&] {
            k_add_scalar(C.T, Y.d() + (size_t)j * B * W, Y.level + 1, B, W, plain_map(), cs, C.stream);
        });
    }
    if (m == 0) return Y;

    // giant steps, then the division tree level by level
    std::vector<DCt> G(m);
    G[0] = std::move(T[k]);
    for (int r = 1; r < m; r++) G[r] = std::move(cheb_steps(C, K, {&G[r - 1]}, {&G[r - 1]}, nullptr)[0]);
    T.clear();
    Tb.clear();
    for (int r = 1; r <= m; r++) {
        const int h = 1 << (m - r);  // parents at this level
        DCt ga;
        const DCt &Ga = aligned(C, G[r - 1], Y.level, ga);
        std::vector<DCt> prods;
        const int per = std::max(1, kChebChunk / B);
        for (int p0 = 0; p0 < h; p0 += per) {
            const int cnt = std::min(per, h - p0);
            std::vector<const DCt *> rep(cnt, &Ga);
            prods.push_back(ev_mul(C, K, slice(C, Y, p0 * B, cnt * B), stack(C, rep)));
        }
        std::vector<const DCt *> pp;
        for (const DCt &d : prods) pp.push_back(&d);
        DCt P = prods.size() == 1 ? std::move(prods[0]) : stack(C, pp);
        DCt S = ev_cmul_to(C, slice(C, Y, h * B, h * B), 1.0, P.level);
        Y = ev_add(C, P, S, false);
    }
    return Y;
}

// a * Cmp on the difference D.  f/g composite: a * (f^{d_f}(g^{d_g}(D)) + 1) / 2
// with the factor a/2 folded into the last polynomial and a/2 added as a
// constant.  Chebyshev: the interpolant's coefficients times a.
static DCt cmp_sign(Ctx &C, const Keys &K, const DCt &D, ckr_sign cmp, double a = 1.0) {
    if (D.level < cmp_levels(cmp)) throw Error{CKR_E_DEPTH, "comparator depth"};
    if (cmp.cheb) {
        std::vector<double> c((size_t)1 << (cmp.cheb - 1));
        cheb_step_coeffs(cmp.cheb, c.data());
        for (double &v : c) v = v * a;
        return cheb_eval(C, K, D, c);
    }
    const int total = cmp.minimax ? cmp.minimax : cmp.d_g + cmp.d_f;
    if (total < 1) throw Error{CKR_E_INVALID, "empty comparator"};
    if (cmp.minimax > kMinimaxStages) throw Error{CKR_E_INVALID, "minimax composite has 5 stages"};
    DCt X;
    const DCt *cur = &D;
    for (int r = 0; r < total; r++) {
        const double *c = cmp.minimax ? kMM[r] : (r < cmp.d_g ? kG : kF);
        double cc[4];
        for (int i = 0; i < 4; i++) cc[i] = (r == total - 1) ? c[i] * (a * 0.5) : c[i];
        X = poly7(C, K, *cur, cc);
        cur = &X;
    }
    return ev_add_const(C, X, a * 0.5);
}

// ------------------------------------------------------------------------
// Rank (Algorithm Rank), argmin (Order Statistic with k = 1 and the
// tie-correction offset), Sorting
// ------------------------------------------------------------------------
static bool sign_valid(ckr_sign c) {
    if (c.cheb) return c.d_g == 0 && c.d_f == 0 && c.minimax == 0 && c.cheb >= 2 && c.cheb <= kChebMaxDepth;
    if (c.minimax) return c.d_g == 0 && c.d_f == 0 && c.minimax <= kMinimaxStages;
    return c.d_g + c.d_f >= 1;
}
static void check_sign(ckr_sign c) {
    if (!sign_valid(c))
        throw Error{CKR_E_INVALID, "empty comparator composition, bad Chebyshev depth or minimax stage count"};
}

static void check_N(const Ctx &C, u32 N) {
    if (N < 2 || (N & (N - 1)) || (u64)N * N > C.n() / 2) throw Error{CKR_E_RANGE, "N must be a power of two with N^2 <= n/2"};
}

// levels: TransR mask, comparator, SumR mask (+ E and E * tie mask with tie-correction)
uint32_t rank_depth(ckr_sign c, int tie) { return 2 + cmp_levels(c) + (tie ? 2 : 0); }

// Rank of N values that are not a power of two (section 3.1): zero-padded to
// the next power of two Np, the comparison matrix masked to its N x N block
// after the comparison so the padding takes part in no comparison; one more
// level.
static int pow2_ceil(int N) {
    int p = 1;
    while (p < N) p <<= 1;
    return p;
}
static void check_N_padded(const Ctx &C, u32 N) {
    const u64 Np = (u64)pow2_ceil((int)N);
    if (N < 2 || Np * Np > C.n() / 2) throw Error{CKR_E_RANGE, "N must be >= 2 with next_pow2(N)^2 <= n/2"};
}
uint32_t rank_depth_n(int N, ckr_sign c, int tie) { return rank_depth(c, tie) + (pow2_ceil(N) != N ? 1 : 0); }
// window of ranks [a, b] (the order statistic is a = b = k): [block mask,]
// TransR mask, comparator, [E, E * tie mask, SumR mask, scaling,] indicator
// (+1 for the two-sided window), O * V, SumC mask
uint32_t order_range_depth(int N, int a, int b, ckr_sign c, ckr_sign i, int tie) {
    return (pow2_ceil(N) != N ? 1 : 0) + 1 + cmp_levels(c) + (tie ? 4 : 0) + ((!tie && i.cheb) ? 1 : 0) +
           cmp_levels(i) + ((a > 1 && b < N) ? 1 : 0) + 2;
}
uint32_t order_stat_depth(int N, int k, ckr_sign c, ckr_sign i, int tie) { return order_range_depth(N, k, k, c, i, tie); }
uint32_t argmin_depth(ckr_sign c, ckr_sign i) { return order_stat_depth(2, 1, c, i, 1); }
// rank, scaling, indicator, indicator product, M * V_R, SumC mask, TransC mask
uint32_t sort_depth(ckr_sign c, ckr_sign i) { return rank_depth(c, 0) + 5 + cmp_levels(i); }

// C = Cmp(V_R, V_C): C[i][j] = Cmp(v_j, v_i)
static DCt cmp_matrix(Ctx &C, const Keys &K, const DCt &V, int N, ckr_sign cmp, DCt *VR_out = nullptr,
                      double a = 1.0) {
    // ReplR runs concurrently with TransR -> ReplC (section 3.1's cost
    // paragraph: the replications run in parallel, so the critical path
    // holds 3 log N rotations instead of 4 log N); the bits are unchanged
    DCt VR, VC;
    {
        Branches br(C);
        br.run([&] { VR = repl_r(C, K, V, N); });
        DCt T = trans_r(C, K, V, N);
        VC = repl_c(C, K, T, N);
        br.join();
    }
    DCt D = ev_cmul_to(C, VR, 1.0, VC.level, &VC, true);  // VR brought to VC's level, minus VC
    if (VR_out) *VR_out = std::move(VR);
    return cmp_sign(C, K, D, cmp, a);
}

static DCt rank(Ctx &C, const Keys &K, const DCt &V, int N, ckr_sign cmp, DCt *VR_out = nullptr) {
    check_N_padded(C, (u32)N);
    check_sign(cmp);
    if ((u32)V.level < rank_depth_n(N, cmp, 0)) throw Error{CKR_E_DEPTH, "not enough levels for rank"};
    const int Np = pow2_ceil(N);
    DCt Cm = cmp_matrix(C, K, V, Np, cmp, VR_out);
    if (Np != N) Cm = ev_mul_plain(C, Cm, get_plain(C, kBlockMask, Np, Cm.level, N));
    DCt S = sum_r(C, K, Cm, Np);
    return ev_add_plain(C, S, get_plain(C, kHalfRow0, N, S.level));
}

// tie-corrected rank k_j = SumR(C + E (delta_{j>=i} - 1/2)), E = C (4 - 4C):
// rank plus the tie-correction offset (their +1/2 and -1/2 cancel), a
// permutation of 1..N with equal values ranked in index order
static DCt tie_rank(Ctx &C, const Keys &K, const DCt &V, int Nr, ckr_sign cmp) {
    check_N_padded(C, (u32)Nr);
    check_sign(cmp);
    if ((u32)V.level < rank_depth_n(Nr, cmp, 1))
        throw Error{CKR_E_DEPTH, "not enough levels for the tie-corrected rank"};
    const int N = pow2_ceil(Nr);  // the layout; Nr < N pads
    DCt Cm = cmp_matrix(C, K, V, N, cmp);
    if (N != Nr) Cm = ev_mul_plain(C, Cm, get_plain(C, kBlockMask, N, Cm.level, Nr));
    DCt w = ev_add_const(C, ev_mul_int(C, Cm, -4), 4.0);
    DCt E = ev_mul(C, K, Cm, w);
    DCt Et = ev_mul_plain(C, E, get_plain(C, kTieMask, N, E.level));
    DCt Ca = ev_cmul_to(C, Cm, 1.0, Et.level);
    return sum_r(C, K, ev_add(C, Ca, Et, false), N);
}

// Multi-Ciphertext Ranking (section 5): L blocks of b values (batch entries of
// Bk).  C_{i,j} = Cmp(ReplR(B_i), ReplC(TransR(B_j))) runs for j >= i only, in
// batched comparator passes of up to kPairChunk pairs; the blocks below the
// diagonal follow from Equation (3), C_{i,j} = (1 - C_{j,i})^T, taken
// column-wise:
//   R_i = TransC(SumC((i - 1) - sum_{j<i} C_{j,i})) + SumR(sum_{j>=i} C_{i,j}) + 1/2
// (1-based i), the SumR term brought down to the TransC term's level.
uint32_t rank_multi_depth(ckr_sign c) { return 3 + cmp_levels(c); }
constexpr int kPairChunk = 32;

static DCt rank_multi(Ctx &C, const Keys &K, const DCt &Bk, int b, ckr_sign cmp) {
    check_N(C, (u32)b);
    check_sign(cmp);
    const int L = Bk.B;
    if (L < 1) throw Error{CKR_E_INVALID, "no blocks"};
    if ((u32)Bk.level < rank_multi_depth(cmp)) throw Error{CKR_E_DEPTH, "not enough levels for the ranking"};
    DCt VR = repl_r(C, K, Bk, b);
    DCt VC = repl_c(C, K, trans_r(C, K, Bk, b), b);
    DCt VRa = ev_cmul_to(C, VR, 1.0, VC.level);
    std::vector<std::pair<int, int>> pairs;
    for (int i = 0; i < L; i++)
        for (int j = i; j < L; j++) pairs.push_back({i, j});
    std::vector<DCt> Srow(L), Tcol(L);
    auto acc = [&](DCt &sum, DCt &&x) { sum = sum.B ? ev_add(C, sum, x, false) : std::move(x); };
    for (size_t p0 = 0; p0 < pairs.size(); p0 += kPairChunk) {
        const size_t np = std::min<size_t>(kPairChunk, pairs.size() - p0);
        std::vector<int> ii, jj;
        for (size_t p = p0; p < p0 + np; p++) ii.push_back(pairs[p].first), jj.push_back(pairs[p].second);
        DCt Cm = cmp_sign(C, K, ev_add(C, gather(C, VRa, ii), gather(C, VC, jj), true), cmp);
        for (size_t p = 0; p < np; p++) {
            const int i = ii[p], j = jj[p];
            acc(Srow[i], slice(C, Cm, (int)p, 1));
            if (j > i) acc(Tcol[j], slice(C, Cm, (int)p, 1));
        }
    }
    std::vector<const DCt *> sp;
    for (const DCt &x : Srow) sp.push_back(&x);
    DCt Rr = sum_r(C, K, stack(C, sp), b);
    DCt R = ev_cmul_to(C, Rr, 1.0, Rr.level - 1);
    if (L > 1) {
        std::vector<DCt> X;
        for (int i = 1; i < L; i++) X.push_back(ev_add_const(C, ev_mul_int(C, Tcol[i], -1), (double)i));
        std::vector<const DCt *> xp;
        for (const DCt &x : X) xp.push_back(&x);
        DCt TC = trans_c(C, K, sum_c(C, K, stack(C, xp), b), b);
        DCt head = slice(C, R, 0, 1), tail = ev_add(C, slice(C, R, 1, L - 1), TC, false);
        R = stack(C, {&head, &tail});
    }
    return ev_add_plain(C, R, get_plain(C, kHalfRow0, b, R.level));
}

// Multi-Ciphertext Sorting (section 5): R = multi-ciphertext ranks; for output
// block i and source block j, M_{i,j} = Ind_0(ReplR(R_j) - (b(i-1)+1 || ... || b i))
// with Ind_0(x) = Cmp(x, -1/2) (1 - Cmp(x, 1/2)) on (x +- 1/2)/N, all L^2
// indicators in one batched comparator pass; S_i = TransC(SumC(sum_j M_{i,j} ReplR(B_j))).
uint32_t sort_multi_depth(ckr_sign c, ckr_sign i) { return rank_multi_depth(c) + 5 + cmp_levels(i); }

static DCt sort_multi(Ctx &C, const Keys &K, const DCt &Bk, int b, ckr_sign cmp, ckr_sign ind) {
    check_N(C, (u32)b);
    check_sign(cmp);
    check_sign(ind);
    const int L = Bk.B;
    if (L < 1) throw Error{CKR_E_INVALID, "no blocks"};
    if ((u32)Bk.level < sort_multi_depth(cmp, ind)) throw Error{CKR_E_DEPTH, "not enough levels for the sort"};
    const double dN = (double)L * (double)b;
    DCt R = rank_multi(C, K, Bk, b, cmp);
    DCt RR = repl_r(C, K, R, b);
    DCt VR = repl_r(C, K, Bk, b);
    // the L^2 (output block, source block) indicators in batched comparator
    // passes of at most kPairChunk ciphertexts: g output blocks at a time
    const int g = std::max(1, kPairChunk / (2 * L));
    std::vector<DCt> Si;
    for (int i0 = 0; i0 < L; i0 += g) {
        const int ng = std::min(g, L - i0), P = ng * L;
        std::vector<DCt> Xi;  // entry (i - i0) * L + j: ReplR(R_j) - steps of output block i
        for (int i = i0; i < i0 + ng; i++) Xi.push_back(ev_add_plain(C, RR, get_plain(C, kStepsBlock, b, RR.level, i)));
        std::vector<const DCt *> xp;
        for (const DCt &x : Xi) xp.push_back(&x);
        DCt Xs = ev_cmul_to(C, stack(C, xp), ind.cheb ? 0.5 / dN : 1.0 / dN, RR.level - 1);
        if (ind.cheb) Xs = ev_plus_conj(C, K, Xs);
        DCt d1 = ev_add_const(C, Xs, 0.5 / dN), d2 = ev_add_const(C, Xs, -0.5 / dN);
        DCt cc = cmp_sign(C, K, stack(C, {&d1, &d2}), ind);
        DCt c1 = slice(C, cc, 0, P), c2 = slice(C, cc, P, P);
        DCt M = ev_mul(C, K, c1, ev_add_const(C, ev_mul_int(C, c2, -1), 1.0));
        std::vector<int> jj;
        for (int i = 0; i < ng; i++)
            for (int j = 0; j < L; j++) jj.push_back(j);
        DCt Pm = ev_mul(C, K, M, ev_cmul_to(C, gather(C, VR, jj), 1.0, M.level));
        for (int i = 0; i < ng; i++) {
            DCt acc = slice(C, Pm, i * L, 1);
            for (int j = 1; j < L; j++) acc = ev_add(C, acc, slice(C, Pm, i * L + j, 1), false);
            Si.push_back(std::move(acc));
        }
    }
    std::vector<const DCt *> sp;
    for (const DCt &x : Si) sp.push_back(&x);
    return trans_c(C, K, sum_c(C, K, stack(C, sp), b), b);
}

// Order statistic k (Algorithm Order Statistic), optionally with the
// tie-correction offset.  The indicator of "the k-th smallest" is one-sided at
// the ends (k = 1: Cmp(1.5, k_j); k = N: Cmp(k_j, N - 1/2); the k_j are
// integral) and the window Cmp(x, -1/2) (1 - Cmp(x, 1/2)) on x = k_j - k
// otherwise, every comparison taken on its argument divided by N.
// Order statistic (section 3.2) over a window of ranks [a, b]; a = b = k is
// the order statistic k, the window [N/2, N/2 + 1] the median of an even N
// (section 4), whose product by 1/2 after the inner product is folded into the
// constant that brings V to the mask's level: value = SumC(O V) / (b - a + 1),
// the mean of the statistics a..b, at no extra level.
// With tie-correction k_j = SumR(C + E (delta_{j>=i} - 1/2)), E = C (4 - 4C)
// (rank plus offset; their +1/2 and -1/2 cancel), a permutation of 1..N.  N
// that is not a power of two pads (section 3.1) and needs tie-correction: the
// padding's k_j are 0, outside every window but a = 1, where V is zero there.
// Without it k_j is the rank SumR(C) + 1/2, the factor +-1/N folded into the
// comparator's last polynomial and no row mask on SumR: the other rows hold
// bounded garbage that O * V annihilates (V is zero outside row 0).
// Indicator: Cmp(b + 1/2, k_j) for a = 1, Cmp(k_j, a - 1/2) for b = N, the
// window Cmp(k_j, a - 1/2) (1 - Cmp(k_j, b + 1/2)) otherwise, every argument
// over N.  onehot = O on the first N slots of row 0; value in slot 0.
static void order_range(Ctx &C, const Keys &K, const DCt &V, int N, int a, int b, int tie, ckr_sign cmp,
                        ckr_sign ind, DCt &onehot, DCt &value) {
    check_N_padded(C, (u32)N);
    check_sign(cmp);
    check_sign(ind);
    const int Np = pow2_ceil(N);  // the layout
    if (a < 1 || a > b || b > N) throw Error{CKR_E_INVALID, "the rank window must satisfy 1 <= a <= b <= N"};
    if (a == 1 && b == N) throw Error{CKR_E_INVALID, "the rank window [1, N] selects every element"};
    if (Np != N && !tie) throw Error{CKR_E_INVALID, "N that is not a power of two needs tie-correction"};
    if ((u32)V.level < order_range_depth(N, a, b, cmp, ind, tie))
        throw Error{CKR_E_DEPTH, "not enough levels for the order statistic"};
    const double dN = (double)N, da = (double)a, db = (double)b;
    const bool lower = a == 1;  // only the upper bound b + 1/2 is tested
    // a Chebyshev indicator takes the real part of its argument (the 1/2 in
    // the scaling); without tie-correction its argument keeps the SumR row
    // mask, so that every slot lies in [-1, 1]
    const bool proj = ind.cheb != 0;
    const double sN = proj ? 2.0 * dN : dN;
    DCt base;  // k_j times -1/N (a = 1) or 1/N
    double off1, off2 = 0.0;
    if (tie) {
        DCt kv = tie_rank(C, K, V, N, cmp);
        base = ev_cmul_to(C, kv, lower ? -1.0 / sN : 1.0 / sN, kv.level - 1);
        if (lower) off1 = (db + 0.5) / dN;
        else off1 = (0.5 - da) / dN, off2 = (-0.5 - db) / dN;
    } else {
        DCt Cm = cmp_matrix(C, K, V, N, cmp, nullptr, lower ? -1.0 / sN : 1.0 / sN);
        base = proj ? sum_r(C, K, Cm, N) : rot_add_chain(C, K, Cm, 0, lg(N), [&](int i) { return (i64)N << i; });
        // SumR(C) = R_j - 1/2
        if (lower) off1 = db / dN;
        else off1 = (1.0 - da) / dN, off2 = -db / dN;
    }
    if (proj) base = ev_plus_conj(C, K, base);
    DCt O;
    if (lower || b == N) {
        O = cmp_sign(C, K, ev_add_const(C, base, off1), ind);
    } else {
        DCt d1 = ev_add_const(C, base, off1), d2 = ev_add_const(C, base, off2);
        // both comparisons in one batched pass
        DCt cc = cmp_sign(C, K, stack(C, {&d1, &d2}), ind);
        const int B = V.B;
        DCt c1 = slice(C, cc, 0, B), c2 = slice(C, cc, B, B);
        O = ev_mul(C, K, c1, ev_add_const(C, ev_mul_int(C, c2, -1), 1.0));
    }
    onehot = ev_mul_plain(C, O, get_plain(C, kMaskRow0, N, O.level));
    DCt Va = ev_cmul_to(C, V, 1.0 / (db - da + 1.0), O.level);
    value = sum_c(C, K, ev_mul(C, K, O, Va), Np);
}

static void order_stat(Ctx &C, const Keys &K, const DCt &V, int N, int k, int tie, ckr_sign cmp, ckr_sign ind,
                       DCt &onehot, DCt &value) {
    check_N(C, (u32)N);
    if (k < 1 || k > N) throw Error{CKR_E_INVALID, "k must lie in [1, N]"};
    order_range(C, K, V, N, k, k, tie, cmp, ind, onehot, value);
}

// Order statistic with the value by division (section 3.2): without
// tie-correction the mask O of rank k may hold several ones (equal values share
// a rank) or none; value = SumC(O V) / SumC(O) by Goldschmidt's iteration on
// the count normalised to x = (2 / (N + 1)) SumC(MaskR(O)) in (0, 2):
//   1/x ~ prod_{i<d} (1 + b^(2^i)),  b = 1 - x  (relative error b^(2^d)),
// the first factor affine, each later one a squaring and a product; then
// value = ((2 / (N + 1)) SumC(O V)) * prod.  d + 2 levels beyond the order
// statistic.
uint32_t order_stat_div_depth(int N, int k, ckr_sign c, ckr_sign i, int iters) {
    return order_stat_depth(N, k, c, i, 0) + iters + 2;
}

static void order_stat_div(Ctx &C, const Keys &K, const DCt &V, int N, int k, ckr_sign cmp, ckr_sign ind, int iters,
                           DCt &onehot, DCt &value) {
    if (iters < 2 || iters > 24) throw Error{CKR_E_INVALID, "Goldschmidt iterations must lie in [2, 24]"};
    check_N(C, (u32)N);
    if (k < 1 || k > N) throw Error{CKR_E_INVALID, "k must lie in [1, N]"};
    if ((u32)V.level < order_stat_div_depth(N, k, cmp, ind, iters))
        throw Error{CKR_E_DEPTH, "not enough levels for the order statistic with division"};
    DCt num;
    order_stat(C, K, V, N, k, 0, cmp, ind, onehot, num);
    const double s = 2.0 / ((double)N + 1.0);
    DCt den = sum_c(C, K, onehot, N);
    DCt x = ev_cmul_to(C, den, s, den.level - 1);
    DCt nx = ev_mul_int(C, x, -1);
    DCt b = ev_add_const(C, nx, 1.0);
    DCt a = ev_add_const(C, nx, 2.0);
    for (int i = 1; i < iters; i++) {
        b = ev_mul(C, K, b, b);
        DCt f = ev_add_const(C, b, 1.0);
        DCt sa;
        const DCt &aa = aligned(C, a, f.level, sa);
        a = ev_mul(C, K, aa, f);
    }
    value = ev_mul(C, K, ev_cmul_to(C, num, s, a.level), a);
}

// Algorithm Sorting: M = Ind_0(ReplR(R) - (1^N || ... || N^N)) with
// Ind_0(x) = Cmp(x, -1/2) (1 - Cmp(x, 1/2)) on (x +- 1/2)/N; S = TransC(SumC(M * ReplR(V)))
static DCt sort(Ctx &C, const Keys &K, const DCt &V, int N, ckr_sign cmp, ckr_sign ind) {
    check_N(C, (u32)N);
    check_sign(cmp);
    check_sign(ind);
    if ((u32)V.level < sort_depth(cmp, ind)) throw Error{CKR_E_DEPTH, "not enough levels for sort"};
    DCt VR;
    DCt R = rank(C, K, V, N, cmp, &VR);
    DCt RR = repl_r(C, K, R, N);
    DCt X = ev_add_plain(C, RR, get_plain(C, kSteps, N, RR.level));
    DCt Xs = ev_cmul_to(C, X, ind.cheb ? 0.5 / (double)N : 1.0 / (double)N, X.level - 1);
    if (ind.cheb) Xs = ev_plus_conj(C, K, Xs);
    DCt d1 = ev_add_const(C, Xs, 0.5 / (double)N);
    DCt d2 = ev_add_const(C, Xs, -0.5 / (double)N);
    // both comparisons in one batched pass
    DCt cc = cmp_sign(C, K, stack(C, {&d1, &d2}), ind);
    const int B = V.B;
    DCt c1 = slice(C, cc, 0, B), c2 = slice(C, cc, B, B);
    DCt M = ev_mul(C, K, c1, ev_add_const(C, ev_mul_int(C, c2, -1), 1.0));
    DCt VRa = ev_cmul_to(C, VR, 1.0, M.level);
    DCt SC = sum_c(C, K, ev_mul(C, K, M, VRa), N);
    return trans_c(C, K, SC, N);
}

// Column-form Sorting (section 3.3, the variant that saves the final
// transposition): the comparator's operands are swapped and SumR becomes SumC,
// so the ranks come out as a column, R'_i = SumC(Cmp(V_C, V_R)) + 1/2 at slot
// i N; rows and columns are then exchanged, with ReplC(TransR(V)) from the
// rank in place of ReplR(V):
//   M = Ind_0(ReplC(R') - (1 || ... || N)^N),  S = SumR(M * ReplC(TransR(V))).
// One level and log N rotations fewer than the row form.
uint32_t sort_col_depth(ckr_sign c, ckr_sign i) { return rank_depth(c, 0) + 4 + cmp_levels(i); }

static DCt sort_col(Ctx &C, const Keys &K, const DCt &V, int N, ckr_sign cmp, ckr_sign ind) {
    check_N(C, (u32)N);
    check_sign(cmp);
    check_sign(ind);
    if ((u32)V.level < sort_col_depth(cmp, ind)) throw Error{CKR_E_DEPTH, "not enough levels for sort"};
    DCt VR = repl_r(C, K, V, N);
    DCt VC = repl_c(C, K, trans_r(C, K, V, N), N);
    DCt D = ev_add(C, VC, ev_cmul_to(C, VR, 1.0, VC.level), true);
    DCt SC = sum_c(C, K, cmp_sign(C, K, D, cmp), N);
    DCt R = ev_add_plain(C, SC, get_plain(C, kHalfCol0, N, SC.level));
    DCt RC = repl_c(C, K, R, N);
    DCt X = ev_add_plain(C, RC, get_plain(C, kStepsCol, N, RC.level));
    DCt Xs = ev_cmul_to(C, X, ind.cheb ? 0.5 / (double)N : 1.0 / (double)N, X.level - 1);
    if (ind.cheb) Xs = ev_plus_conj(C, K, Xs);
    DCt d1 = ev_add_const(C, Xs, 0.5 / (double)N);
    DCt d2 = ev_add_const(C, Xs, -0.5 / (double)N);
    // both comparisons in one batched pass
    DCt cc = cmp_sign(C, K, stack(C, {&d1, &d2}), ind);
    const int B = V.B;
    DCt c1 = slice(C, cc, 0, B), c2 = slice(C, cc, B, B);
    DCt M = ev_mul(C, K, c1, ev_add_const(C, ev_mul_int(C, c2, -1), 1.0));
    DCt VCa = ev_cmul_to(C, VC, 1.0, M.level);
    return sum_r(C, K, ev_mul(C, K, M, VCa), N);
}

enum CircuitKind { kRankCircuit = 1, kArgminCircuit = 2, kSortCircuit = 3, kOrderCircuit = 4, kSortColCircuit = 5 };

// levels a circuit consumes
static uint32_t spec_depth(const Spec &s) {
    if (s.kind == kRankCircuit) return rank_depth_n(s.N, s.cmp, s.tie);
    if (s.kind == kSortCircuit) return sort_depth(s.cmp, s.ind);
    if (s.kind == kSortColCircuit) return sort_col_depth(s.cmp, s.ind);
    return order_range_depth(s.N, s.k, s.k_hi, s.cmp, s.ind, s.tie);
}

// the circuit of a (kind, N, compositions) request; argmin is the
// tie-corrected order statistic k = 1
static Spec spec_of(const Ctx &C, int kind, int N, int k, int tie, ckr_sign cmp, ckr_sign ind) {
    if (kind == kRankCircuit) check_N_padded(C, (u32)N);
    else check_N(C, (u32)N);
    Spec s;
    s.N = N;
    s.cmp = cmp;
    if (kind == kRankCircuit) {
        s.kind = kind;
        s.tie = tie != 0;
    } else if (kind == kSortCircuit || kind == kSortColCircuit) {
        s.kind = kind;
        s.ind = ind;
    } else if (kind == kArgminCircuit || kind == kOrderCircuit) {
        s.kind = kOrderCircuit;
        s.k = s.k_hi = kind == kArgminCircuit ? 1 : k;
        s.tie = kind == kArgminCircuit ? 1 : (tie != 0);
        s.ind = ind;
        if (s.k < 1 || s.k > N) throw Error{CKR_E_INVALID, "k must lie in [1, N]"};
    } else {
        throw Error{CKR_E_INVALID, "unknown circuit kind"};
    }
    if (!sign_valid(s.cmp) || (s.kind != kRankCircuit && !sign_valid(s.ind)))
        throw Error{CKR_E_INVALID, "empty comparator"};
    return s;
}

static std::vector<DCt> eval_spec(Ctx &C, const Keys &K, const Spec &s, const DCt &X) {
    std::vector<DCt> o;
    if (s.kind == kRankCircuit) {
        o.push_back(s.tie ? tie_rank(C, K, X, s.N, s.cmp) : rank(C, K, X, s.N, s.cmp));
    } else if (s.kind == kSortCircuit) {
        o.push_back(sort(C, K, X, s.N, s.cmp, s.ind));
    } else if (s.kind == kSortColCircuit) {
        o.push_back(sort_col(C, K, X, s.N, s.cmp, s.ind));
    } else {
        o.resize(2);
        order_range(C, K, X, s.N, s.k, s.k_hi, s.tie, s.cmp, s.ind, o[0], o[1]);
    }
    return o;
}

// Run query groups (each a circuit on a batch of single ciphertexts of one
// level) as one unit.  With graphs enabled, the first call for a plan runs
// eagerly (filling plaintext and table caches), the second captures every
// group's circuit into one hipGraph, later calls copy the inputs into the
// plan's input batches and replay it with a single launch.  Every path
// launches the same kernels in the same order: outputs are bit-identical.
using Circuit = std::function<std::vector<DCt>(const std::vector<DCt> &)>;

constexpr int kPlansPerSlot = 16;

static std::vector<DCt> run_circuit(Ctx &C, Keys &K, const PlanKey &key,
                                    const std::vector<std::vector<const DCt *>> &in, const Circuit &circuit) {
    auto fill = [&](std::vector<DCt> &X) {
        for (size_t g = 0; g < key.size(); g++) {
            const size_t W = (size_t)2 * (key[g].level + 1) * C.n();
            for (int i = 0; i < key[g].B; i++)
                HIPCHK(hipMemcpyAsync(X[g].d() + i * W, in[g][i]->d(), W * 8, hipMemcpyDeviceToDevice, C.stream));
        }
    };
    auto inputs = [&] {
        std::vector<DCt> X;
        for (const GroupKey &g : key) X.push_back(ct_new(C, g.level, g.B));
        return X;
    };
    const bool use_graph = C.graphs && !C.prof.on;
    auto it = K.plans.find({C.slot, key});
    if (it != K.plans.end() && it->second->epoch != C.tune_epoch) {
        // captured with other tiles or chunking: capture again, so that a
        // replay always runs the kernels the context is set to
        K.plans.erase(it);
        it = K.plans.end();
    }
    if (!use_graph || (it == K.plans.end() && !K.warm.count(key))) {
        std::vector<DCt> X = inputs();
        fill(X);
        std::vector<DCt> outs = circuit(X);
        K.warm.insert(key);
        return outs;
    }
    if (it == K.plans.end()) {
        // at most kPlansPerSlot captured plans per slot: each holds its
        // temporaries until destroyed, so a new batch size or level past the
        // cap evicts the slot's least recently replayed plan (this slot's
        // plans only run on this thread; the destructor waits for the stream)
        int mine = 0;
        auto lru = K.plans.end();
        for (auto p = K.plans.begin(); p != K.plans.end(); ++p)
            if (p->first.first == C.slot) {
                mine++;
                if (lru == K.plans.end() || p->second->last_use < lru->second->last_use) lru = p;
            }
        if (mine >= kPlansPerSlot) K.plans.erase(lru);
        auto plan = std::make_unique<GraphPlan>();
        plan->C = &C;
        plan->stream = C.stream;
        plan->epoch = C.tune_epoch;
        plan->in = inputs();
        sync(C);
        HIPCHK(hipStreamBeginCapture(C.stream, hipStreamCaptureModeRelaxed));
        C.pool.begin_capture();
        try {
            plan->outs = circuit(plan->in);
        } catch (...) {
            plan->owned = C.pool.end_capture();
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(C.stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        plan->owned = C.pool.end_capture();
        HIPCHK(hipStreamEndCapture(C.stream, &plan->graph));
        HIPCHK(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
        it = K.plans.emplace(std::make_pair(C.slot, key), std::move(plan)).first;
    }
    GraphPlan &pl = *it->second;
    pl.last_use = ++K.plan_clock;
    fill(pl.in);
    HIPCHK(hipGraphLaunch(pl.exec, C.stream));
    std::vector<DCt> outs;
    for (const DCt &o : pl.outs) outs.push_back(slice(C, o, 0, o.B));
    return outs;
}

// groups[g] runs specs[g] on the single ciphertexts in[g] (all of one level);
// returns each group's batched outputs
static std::vector<std::vector<DCt>> run_groups(Ctx &C, Keys &K, const std::vector<Spec> &specs,
                                                const std::vector<std::vector<const DCt *>> &in) {
    PlanKey key;
    for (size_t g = 0; g < specs.size(); g++) {
        if (in[g].empty()) throw Error{CKR_E_INVALID, "empty batch"};
        const int level = in[g][0]->level;
        for (auto *c : in[g])
            if (c->level != level || c->B != 1)
                throw Error{CKR_E_INVALID, "batch entries must be single ciphertexts of one level"};
        if ((u32)level < spec_depth(specs[g])) throw Error{CKR_E_DEPTH, "not enough levels for the circuit"};
        if (level > K.lmax) throw Error{CKR_E_DEPTH, "ciphertext above key level"};
        key.push_back(GroupKey{specs[g], level, (int)in[g].size()});
    }
    Circuit f = [&](const std::vector<DCt> &X) {
        // the groups are independent circuits: each runs as a branch on a side
        // stream (their own replication branches then run inline: branches do
        // not nest), joined before the outputs are used
        std::vector<std::vector<DCt>> per(specs.size());
        if (specs.size() > 1) {
            Branches br(C);
            for (size_t g = 0; g < specs.size(); g++) br.run([&, g] { per[g] = eval_spec(C, K, specs[g], X[g]); });
            br.join();
        } else {
            per[0] = eval_spec(C, K, specs[0], X[0]);
        }
        std::vector<DCt> outs;
        for (auto &v : per)
            for (DCt &o : v) outs.push_back(std::move(o));
        return outs;
    };
    std::vector<DCt> flat = run_circuit(C, K, key, in, f);
    std::vector<std::vector<DCt>> res(specs.size());
    size_t pos = 0;
    for (size_t g = 0; g < specs.size(); g++) {
        const int per = specs[g].kind == kOrderCircuit ? 2 : 1;
        for (int j = 0; j < per; j++) res[g].push_back(std::move(flat[pos++]));
    }
    return res;
}

static std::vector<DCt> run_kind(Ctx &C, Keys &K, int kind, int N, ckr_sign cmp, ckr_sign ind,
                                 const std::vector<const DCt *> &in) {
    const Spec s = spec_of(C, kind, N, 1, kind == kArgminCircuit, cmp, ind);
    std::vector<std::vector<DCt>> r = run_groups(C, K, {s}, {in});
    return std::move(r[0]);
}

// ------------------------------------------------------------------------
// serving: continuous batching over a request queue with HBM admission
// ------------------------------------------------------------------------
static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Route {
    int kind, N;
    Ctx *C;
    Keys *K;
    ckr_sign cmp, ind;
    size_t bytes_per_query = 0;  // measured on the route's first batch
};

struct Request {
    u64 ticket;
    int route;
    const DCt *in;  // caller-owned, alive until the ticket completes
    double t_submit = 0, t_start = 0, t_done = 0;
    std::vector<DCt> outs;
    int status = CKR_OK;
    std::string err;
    bool done = false;
    int batch = 0;
};

class Server {
  public:
    Server(size_t budget, int max_batch) : budget_(budget), max_batch_(std::max(1, max_batch)) {}
    ~Server() { stop(); }

    int add_route(const Route &r) {
        std::lock_guard<std::mutex> g(mu_);
        if (started_) throw Error{CKR_E_BUSY, "routes must be added before the first submit"};
        routes_.push_back(r);
        return (int)routes_.size() - 1;
    }

    u64 submit(int kind, int N, const DCt &v) {
        std::lock_guard<std::mutex> g(mu_);
        int route = -1;
        for (size_t i = 0; i < routes_.size(); i++)
            if (routes_[i].kind == kind && routes_[i].N == N) route = (int)i;
        if (route < 0) throw Error{CKR_E_INVALID, "no route for this circuit and N"};
        if (v.B != 1) throw Error{CKR_E_INVALID, "submit one ciphertext"};
        auto rq = std::make_unique<Request>();
        rq->route = route;
        rq->in = &v;
        rq->t_submit = now_ms();
        start_locked();
        const u64 t = ++next_ticket_;
        rq->ticket = t;
        pending_.push_back(t);
        reqs_[t] = std::move(rq);
        cv_.notify_all();
        return t;
    }

    // waits for the ticket; moves its outputs out and forgets it
    int wait(u64 ticket, int timeout_ms, std::vector<DCt> &outs, double *lat_ms, std::string &err, Ctx **ctx) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) throw Error{CKR_E_INVALID, "unknown ticket"};
        Request *r = it->second.get();
        auto ready = [&] { return r->done; };
        if (timeout_ms < 0) cv_.wait(lk, ready);
        else if (!cv_.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) return CKR_E_BUSY;
        if (lat_ms) {
            lat_ms[0] = r->t_done - r->t_submit;
            lat_ms[1] = r->t_start - r->t_submit;
            lat_ms[2] = (double)r->batch;
        }
        const int st = r->status;
        err = r->err;
        outs = std::move(r->outs);
        *ctx = routes_[r->route].C;
        std::unique_ptr<Request> keep = std::move(it->second);
        reqs_.erase(it);
        lk.unlock();
        return st;
    }

    void stats(double *out) {
        std::lock_guard<std::mutex> g(mu_);
        out[0] = (double)completed_;
        out[1] = (double)batches_;
        out[2] = (double)inflight_high_;
        out[3] = (double)pending_.size();
        out[4] = (double)overlap_high_;
    }

    void stop() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
            cv_.notify_all();
        }
        for (auto &t : workers_) t.join();
        workers_.clear();
        for (Ctx *c : ctxs_) c->pool.set_local(false);
        ctxs_.clear();
        // requests that never ran complete with an error, so no wait blocks forever
        std::lock_guard<std::mutex> g(mu_);
        for (u64 t : pending_) {
            Request *r = reqs_[t].get();
            r->status = CKR_E_INVALID;
            r->err = "server stopped before the request ran";
            r->t_done = now_ms();
            r->done = true;
        }
        pending_.clear();
        cv_.notify_all();
    }

  private:
    static std::recursive_mutex &ctx_mu(Ctx *C) { return C->mu_run; }

    // Each context gets Ctx::kSlots workers, each issuing its batches on a
    // stream of its own: a request that arrives while a batch of its context
    // runs starts in the next free slot (admission permitting), so batches of
    // one context overlap on the device.  The pool then reuses a freed block
    // only on the stream that freed it until the host has waited for it.
    void start_locked() {
        if (started_) return;
        started_ = true;
        for (auto &r : routes_)
            if (std::find(ctxs_.begin(), ctxs_.end(), r.C) == ctxs_.end()) ctxs_.push_back(r.C);
        for (Ctx *c : ctxs_) {
            c->pool.set_local(true);
            for (int s = 1; s <= Ctx::kSlots; s++) workers_.emplace_back([this, c, s] { work(c, s); });
        }
    }

    // oldest pending request of this context, then up to max_batch of the same route and level
    bool pick(Ctx *C, std::vector<Request *> &batch, size_t &bytes) {
        batch.clear();
        if (exclusive_[C]) return false;  // a route's measuring batch runs alone on its context
        Request *first = nullptr;
        for (u64 t : pending_) {
            Request *r = reqs_[t].get();
            if (routes_[r->route].C == C) {
                first = r;
                break;
            }
        }
        if (!first) return false;
        const Route &rt = routes_[first->route];
        if (!rt.bytes_per_query && active_[C] > 0) return false;  // measure alone
        int cap = rt.bytes_per_query ? max_batch_ : 1;  // first batch of a route measures its working set
        for (u64 t : pending_) {
            Request *r = reqs_[t].get();
            if ((int)batch.size() < cap && r->route == first->route && r->in->level == first->in->level) batch.push_back(r);
        }
        const size_t per = rt.bytes_per_query;
        if (budget_ && per) {
            while (!batch.empty() && inflight_ + per * batch.size() > budget_) batch.pop_back();
            if (batch.empty()) {
                if (inflight_ == 0) {  // one query alone does not fit: fail it
                    first->status = CKR_E_NOMEM;
                    first->err = "request exceeds the HBM budget";
                    first->done = true;
                    first->t_done = now_ms();
                    pending_.erase(std::find(pending_.begin(), pending_.end(), first->ticket));
                    cv_.notify_all();
                }
                return false;
            }
        }
        bytes = per * batch.size();
        return true;
    }

    void work(Ctx *C, int slot) {
        HIPCHK_NOTHROW(hipSetDevice(C->device));
        hipEvent_t done_ev = nullptr;
        HIPCHK_NOTHROW(hipEventCreateWithFlags(&done_ev, hipEventDisableTiming));
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            std::vector<Request *> batch;
            size_t bytes = 0;
            cv_.wait(lk, [&] { return stop_ || pick(C, batch, bytes); });
            if (stop_ && batch.empty()) break;
            for (Request *r : batch) pending_.erase(std::find(pending_.begin(), pending_.end(), r->ticket));
            inflight_ += bytes;
            inflight_high_ = std::max(inflight_high_, inflight_);
            const Route rt = routes_[batch[0]->route];
            const bool measure = rt.bytes_per_query == 0;
            if (measure) exclusive_[C] = true;
            overlap_high_ = std::max(overlap_high_, ++active_[C]);
            lk.unlock();
            const double t0 = now_ms();
            std::vector<std::vector<DCt>> per(batch.size());
            int st = CKR_OK;
            std::string err;
            size_t measured = 0;
            hipStream_t sst = nullptr;
            try {
                {
                    // enqueue under the context lock on this slot's stream, wait outside it
                    std::lock_guard<std::recursive_mutex> cg(ctx_mu(C));
                    C->ensure_slot(slot);
                    sst = C->slot_stream[slot];
                    struct Use {
                        Ctx *C;
                        hipStream_t s0;
                        int k0;
                        ~Use() {
                            C->stream = s0;
                            C->slot = k0;
                        }
                    } use{C, C->stream, C->slot};
                    C->stream = sst;
                    C->slot = slot;
                    const size_t base = C->pool.in_use;
                    if (measure) C->pool.high = base;
                    std::vector<const DCt *> in;
                    for (Request *r : batch) in.push_back(r->in);
                    // the measuring batch runs eagerly so the pool sees its whole working set
                    const bool graphs = C->graphs;
                    if (measure) C->graphs = false;
                    std::vector<DCt> outs;
                    try {
                        outs = run_kind(*C, *rt.K, rt.kind, rt.N, rt.cmp, rt.ind, in);
                    } catch (...) {
                        C->graphs = graphs;
                        throw;
                    }
                    C->graphs = graphs;
                    for (size_t i = 0; i < batch.size(); i++)
                        for (auto &o : outs) per[i].push_back(slice(*C, o, (int)i, 1));
                    outs.clear();  // freed on this slot's stream
                    if (measure) measured = (C->pool.high - base) / batch.size();
                    HIPCHK(hipEventRecord(done_ev, sst));
                }
                HIPCHK(hipEventSynchronize(done_ev));
                C->pool.flush(sst);
            } catch (const Error &e) {
                st = e.status;
                err = e.msg;
            } catch (const std::exception &e) {
                st = CKR_E_INVALID;
                err = e.what();
            }
            if (st != CKR_OK && sst) {
                // the batch's work may still be queued: wait before its blocks serve other streams
                (void)hipStreamSynchronize(sst);
                C->pool.flush(sst);
            }
            const double t1 = now_ms();
            lk.lock();
            if (measure && measured) routes_[batch[0]->route].bytes_per_query = measured;
            if (measure) exclusive_[C] = false;
            active_[C]--;
            inflight_ -= bytes;
            for (size_t i = 0; i < batch.size(); i++) {
                Request *r = batch[i];
                r->status = st;
                r->err = err;
                if (st == CKR_OK) r->outs = std::move(per[i]);
                r->t_start = t0;
                r->t_done = t1;
                r->batch = (int)batch.size();
                r->done = true;
            }
            completed_ += batch.size();
            batches_++;
            cv_.notify_all();
        }
        if (done_ev) (void)hipEventDestroy(done_ev);
    }

    std::mutex mu_;
    std::condition_variable cv_;
    std::vector<Route> routes_;
    std::deque<u64> pending_;
    std::unordered_map<u64, std::unique_ptr<Request>> reqs_;
    std::vector<std::thread> workers_;
    size_t budget_, inflight_ = 0, inflight_high_ = 0;
    std::vector<Ctx *> ctxs_;
    std::map<Ctx *, int> active_;      // batches of each context in flight
    std::map<Ctx *, bool> exclusive_;  // a measuring batch runs on the context
    int overlap_high_ = 0;             // most batches of one context in flight at once
    int max_batch_;
    u64 next_ticket_ = 0, completed_ = 0, batches_ = 0;
    bool stop_ = false, started_ = false;
};

}  // namespace ckr

// ========================================================================
// C ABI
// ========================================================================
using namespace ckr;

struct ckr_context {
    std::unique_ptr<Ctx> C;
};
struct ckr_keys {
    std::unique_ptr<Keys> K;
};
struct ckr_ct {
    Ctx *C;
    DCt ct;
};

// ------------------------------------------------------------------------
// scratch memory of the allocation-free rotation (ckr_op_rotate_into)
// ------------------------------------------------------------------------
// A file-scope device array: every GPU the library runs on holds its own copy
// at its own address until the process ends.  In host code `scratch` names a
// host-side stand-in, so its device address is looked up once per device
// (with that device current) and only that address is ever handed to kernels.
constexpr size_t kScratchWords = size_t(16) << 20;  // 128 MiB
static __device__ __align__(256) u64 scratch[kScratchWords];
static std::mutex g_scratch_mu;
static std::map<int, u64 *> g_scratch_dev;

static u64 *scratch_ptr(int dev) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_dev.find(dev);
    if (it != g_scratch_dev.end()) return it->second;
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error{CKR_E_DEVICE, "no device address for the scratch array"};
    g_scratch_dev[dev] = (u64 *)p;
    return (u64 *)p;
}

// words of scratch one key switch of a single ciphertext at level l takes:
// the coefficient-domain input, the extended digits, the two accumulators
// and the ModDown conversion (each block 256-byte aligned)
static size_t keyswitch_scratch_words(const Ctx &C, int l) {
    const size_t n = C.n(), E = (size_t)(l + 1 + C.P.K), beta = (size_t)C.P.beta(l);
    auto al = [](size_t w) { return (w + 31) & ~size_t(31); };
    return al((size_t)(l + 1) * n) + al(beta * E * n) + al(2 * E * n) + al((size_t)2 * (l + 1) * n);
}

template <class F>
static ckr_status guard(F &&f) {
    try {
        f();
        return CKR_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return (ckr_status)e.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return CKR_E_NOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return CKR_E_INVALID;
    } catch (...) {
        g_last_error = "unknown error";
        return CKR_E_INVALID;
    }
}

#define NEED(x)                                                   \
    do {                                                          \
        if (!(x)) throw Error{CKR_E_INVALID, "null argument: " #x}; \
    } while (0)

extern "C" {

const char *ckr_last_error(void) { return g_last_error.c_str(); }

ckr_status ckr_context_create(const ckr_params *p, int dev, size_t budget, ckr_context **out) {
    return guard([&] {
        NEED(p && out);
        *out = nullptr;
        int count = 0;
        HIPCHK(hipGetDeviceCount(&count));
        if (dev < 0 || dev >= count) throw Error{CKR_E_DEVICE, "no such HIP device"};
        HIPCHK(hipSetDevice(dev));
        auto ctx = std::make_unique<ckr_context>();
        ctx->C = std::make_unique<Ctx>();
        Ctx &C = *ctx->C;
        C.device = dev;
        C.P = make_params((int)p->log_n, (int)p->n_q, (int)p->q0_bits, (int)p->log_scale, (int)p->n_p,
                          (int)p->p_bits, (int)p->dnum);
        if (C.P.alpha > kMaxBConvSrc || C.P.K > kMaxBConvSrc) throw Error{CKR_E_INVALID, "digit too large"};
        if (C.P.dnum > 8) throw Error{CKR_E_INVALID, "at most 8 key-switching digits"};
        if (C.P.nmod() > kMaxLimbArgs) throw Error{CKR_E_INVALID, "too many primes"};
        C.pool.budget = budget;
        setup_tables(C);
        C.scratch = scratch_ptr(dev);
        // a stream of the context's own (default priority): graph capture needs a non-null stream
        HIPCHK(hipStreamCreate(&C.own_stream));
        C.stream = C.own_stream;
        for (hipStream_t &st : C.side[0]) HIPCHK(hipStreamCreate(&st));
        C.pool.set_cur((const void *const *)&C.stream);
        *out = ctx.release();
    });
}

void ckr_context_free(ckr_context *ctx) { delete ctx; }

ckr_status ckr_context_set_stream(ckr_context *ctx, void *s) {
    return guard([&] {
        NEED(ctx);
        ctx->C->stream = (hipStream_t)s;
    });
}

ckr_status ckr_context_set_allocator(ckr_context *ctx, void *(*a)(size_t, void *), void (*f)(void *, void *),
                                     void *user) {
    return guard([&] {
        NEED(ctx && a && f);
        if (ctx->C->pool.held) throw Error{CKR_E_INVALID, "allocator must be set before any allocation"};
        ctx->C->pool.ualloc = a;
        ctx->C->pool.ufree = f;
        ctx->C->pool.user = user;
    });
}

ckr_status ckr_context_info(const ckr_context *ctx, uint64_t *mods, double *scales) {
    return guard([&] {
        NEED(ctx);
        const Params &P = ctx->C->P;
        if (mods) std::copy(P.mod.begin(), P.mod.end(), mods);
        if (scales) std::copy(P.scale.begin(), P.scale.end(), scales);
    });
}

ckr_status ckr_params_derive(const ckr_params *p, uint64_t *mods, double *scales) {
    return guard([&] {
        NEED(p);
        Params P = make_params((int)p->log_n, (int)p->n_q, (int)p->q0_bits, (int)p->log_scale, (int)p->n_p,
                               (int)p->p_bits, (int)p->dnum);
        if (mods) std::copy(P.mod.begin(), P.mod.end(), mods);
        if (scales) std::copy(P.scale.begin(), P.scale.end(), scales);
    });
}

ckr_status ckr_encode(uint32_t log_n, const double *z, uint32_t count, double scale, int64_t *m) {
    return guard([&] {
        NEED(z && m);
        if (log_n < 10 || log_n > 17) throw Error{CKR_E_INVALID, "log_n must be in [10, 17]"};
        if ((u64)count > (1ull << log_n) / 2) throw Error{CKR_E_RANGE, "too many slots"};
        if (!encode_slots((int)log_n, z, count, scale, m)) throw Error{CKR_E_RANGE, "coefficient overflow"};
    });
}

ckr_status ckr_sample(const uint8_t seed[32], uint32_t purpose, uint64_t id, int kind, uint64_t q, size_t count,
                      int64_t *out) {
    return guard([&] {
        NEED(seed && out);
        if (kind == 2 && q < 2) throw Error{CKR_E_INVALID, "modulus"};
        Stream st(seed, purpose, id);
        for (size_t i = 0; i < count; i++)
            out[i] = kind == 0 ? st.ternary() : kind == 1 ? st.cbd21() : (int64_t)st.uniform(q);
    });
}

ckr_status ckr_context_memory(const ckr_context *ctx, size_t *in_use, size_t *high) {
    return guard([&] {
        NEED(ctx);
        if (in_use) *in_use = ctx->C->pool.in_use;
        if (high) *high = ctx->C->pool.high;
    });
}

// run fn(i) for i in [0, count) on up to 16 host threads (independent streams per i)
static void parallel_for(int count, const std::function<void(int)> &fn) {
    const int T = std::max(1, std::min<int>({count, 16, (int)std::thread::hardware_concurrency()}));
    if (T <= 1) {
        for (int i = 0; i < count; i++) fn(i);
        return;
    }
    std::vector<std::thread> th;
    std::atomic<int> next{0};
    for (int t = 0; t < T; t++)
        th.emplace_back([&] {
            for (int i = next++; i < count; i = next++) fn(i);
        });
    for (auto &x : th) x.join();
}

// Galois elements the circuits need for one N
static void circuit_shifts(u32 Nr, u32 what, std::vector<i64> &sh) {
    const u32 N = (u32)pow2_ceil((int)Nr);  // a padded rank uses the next power of two's layout
    const int l = lg((int)N);
    for (int i = 1; i <= l; i++) sh.push_back(-(i64)(((i64)N * (N - 1)) >> i));  // TransR
    for (int i = 0; i < l; i++) sh.push_back(-((i64)N << i));                     // ReplR
    for (int i = 0; i < l; i++) sh.push_back(-((i64)1 << i));                     // ReplC
    for (int i = 0; i < l; i++) sh.push_back((i64)N << i);                        // SumR
    if (what & 6) {
        for (int i = 0; i < l; i++) sh.push_back((i64)1 << i);                    // SumC
    }
    if (what & 4) {
        for (int i = 1; i <= l; i++) sh.push_back((i64)(((i64)N * (N - 1)) >> i));  // TransC
    }
}

// switching key for target s' (eval domain, limbs of (q_0..q_lmax, P)):
//   b_j = -a_j s + e_j + [limb in digit j] (P mod q) s',  a_j uniform
static void gen_switch_key(Ctx &C, Keys &K, u32 g, const Buf &s_eval, const Buf &sp_eval, const uint8_t *seed) {
    const Params &P = C.P;
    const size_t n = C.n();
    const int Ek = K.Ek(), beta = P.beta(K.lmax);
    Buf key(&C, (size_t)beta * 2 * Ek * n);
    const LimbMap emap{K.lmax + 1, 0, P.nq};
    std::vector<u64> a((size_t)Ek * n), e((size_t)Ek * n);
    Buf ea(&C, (size_t)Ek * n), ee(&C, (size_t)Ek * n), tmp(&C, (size_t)Ek * n);
    for (int j = 0; j < beta; j++) {
        std::vector<i64> ei(n);
        {
            Stream st(seed, kKsE, ((u64)g << 32) | ((u64)j << 16));
            for (size_t i = 0; i < n; i++) ei[i] = st.cbd21();
        }
        parallel_for(Ek, [&](int li) {
            const int mt = emap(li);
            const u64 q = P.mod[mt];
            Stream st(seed, kKsA, ((u64)g << 32) | ((u64)j << 16) | (u64)mt);
            u64 *ar = a.data() + (size_t)li * n, *er = e.data() + (size_t)li * n;
            for (size_t i = 0; i < n; i++) ar[i] = st.uniform(q);
            for (size_t i = 0; i < n; i++) er[i] = hred(ei[i], q);
        });
        HIPCHK(hipMemcpyAsync(ea.get(), a.data(), a.size() * 8, hipMemcpyHostToDevice, C.stream));
        HIPCHK(hipMemcpyAsync(ee.get(), e.data(), e.size() * 8, hipMemcpyHostToDevice, C.stream));
        ntt(C, ea.get(), Ek, 1, 0, emap, false);
        ntt(C, ee.get(), Ek, 1, 0, emap, false);
        u64 *kb = key.get() + (size_t)(j * 2) * Ek * n, *ka = kb + (size_t)Ek * n;
        // kb = e - a*s
        k_mul_pt(C.T, tmp.get(), ea.get(), s_eval.get(), Ek, 1, 0, 0, emap, false, C.stream);
        k_add(C.T, kb, ee.get(), tmp.get(), Ek, 1, 0, 0, 0, emap, true, C.stream);
        // + (P mod q) s' on the limbs of digit j
        const int lo = j * P.alpha, hi = std::min(lo + P.alpha, K.lmax + 1) - 1;
        std::vector<u64> pm;
        for (int i = lo; i <= hi; i++) {
            u64 pp = 1 % P.mod[i];
            for (int k = 0; k < P.K; k++) pp = hmul(pp, P.mod[P.nq + k] % P.mod[i], P.mod[i]);
            pm.push_back(pp);
        }
        LimbScalars sc;
        for (size_t i = 0; i < pm.size(); i++) {
            sc.v[i] = (double)pm[i];
            sc.vq[i] = (double)pm[i] / (double)P.mod[lo + i];
        }
        k_mul_scalar(C.T, tmp.get(), sp_eval.get() + (size_t)lo * n, hi - lo + 1, 1, 0, 0, plain_map(lo), sc, C.stream);
        k_add(C.T, kb + (size_t)lo * n, kb + (size_t)lo * n, tmp.get(), hi - lo + 1, 1, 0, 0, 0, plain_map(lo), false,
              C.stream);
        HIPCHK(hipMemcpyAsync(ka, ea.get(), (size_t)Ek * n * 8, hipMemcpyDeviceToDevice, C.stream));
        sync(C);  // host staging reused next digit
    }
    K.swk[g] = std::move(key);
}

static void add_galois_keys(Ctx &C, Keys &K, const std::vector<u32> &gals, const uint8_t *seed) {
    const size_t n = C.n();
    const int Ek = K.Ek();
    const LimbMap emap{K.lmax + 1, 0, C.P.nq};
    // secret in eval domain on (q_0..q_lmax, P)
    std::vector<u64> sr((size_t)Ek * n);
    for (int li = 0; li < Ek; li++)
        for (size_t i = 0; i < n; i++) sr[(size_t)li * n + i] = hred(K.s[i], C.P.mod[emap(li)]);
    Buf s_eval(&C, sr.size());
    HIPCHK(hipMemcpyAsync(s_eval.get(), sr.data(), sr.size() * 8, hipMemcpyHostToDevice, C.stream));
    ntt(C, s_eval.get(), Ek, 1, 0, emap, false);
    Buf sp(&C, sr.size());
    for (u32 g : gals) {
        if (g == 1 || K.swk.count(g)) continue;
        k_automorph(C.T, sp.get(), s_eval.get(), Ek, 1, 0, 0, g, C.stream);
        gen_switch_key(C, K, g, s_eval, sp, seed);
    }
    sync(C);
}

static void add_rotation_keys(Ctx &C, Keys &K, const std::vector<i64> &shifts, const uint8_t *seed) {
    std::vector<u32> gals;
    for (i64 k : shifts) gals.push_back(galois_left(C, k));
    add_galois_keys(C, K, gals, seed);
}

static std::map<const Keys *, std::vector<uint8_t>> g_key_seed;  // seeds kept for later rotation keys
static std::mutex g_key_seed_mu;

ckr_status ckr_keygen(ckr_context *ctx, const uint8_t seed[32], uint32_t max_level, const uint32_t *Ns, size_t nN,
                      uint32_t what, ckr_keys **out) {
    return guard([&] {
        NEED(ctx && seed && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = nullptr;
        Ctx &C = *ctx->C;
        const Params &P = C.P;
        if ((int)max_level > P.L) throw Error{CKR_E_DEPTH, "max_level above the chain"};
        for (size_t i = 0; i < nN; i++) check_N_padded(C, Ns[i]);  // keys of the padded layout
        auto K = std::make_unique<Keys>();
        K->C = &C;
        K->lmax = (int)max_level;
        const size_t n = C.n();
        K->s.resize(n);
        {
            Stream st(seed, kSecret, 0);
            for (size_t i = 0; i < n; i++) K->s[i] = st.ternary();
        }
        const int Ek = K->Ek();
        const LimbMap emap{K->lmax + 1, 0, P.nq};
        std::vector<u64> sr((size_t)Ek * n);
        for (int li = 0; li < Ek; li++)
            for (size_t i = 0; i < n; i++) sr[(size_t)li * n + i] = hred(K->s[i], P.mod[emap(li)]);
        Buf s_eval(&C, sr.size());
        HIPCHK(hipMemcpyAsync(s_eval.get(), sr.data(), sr.size() * 8, hipMemcpyHostToDevice, C.stream));
        ntt(C, s_eval.get(), Ek, 1, 0, emap, false);
        // public key on q_0..q_lmax: (e - a s, a)
        {
            const int L1 = K->lmax + 1;
            std::vector<i64> e(n);
            {
                Stream st(seed, kPkE, 0);
                for (size_t i = 0; i < n; i++) e[i] = st.cbd21();
            }
            std::vector<u64> a((size_t)L1 * n), er((size_t)L1 * n);
            for (int t = 0; t < L1; t++) {
                Stream st(seed, kPkA, (u64)t);
                for (size_t i = 0; i < n; i++) a[(size_t)t * n + i] = st.uniform(P.mod[t]);
                for (size_t i = 0; i < n; i++) er[(size_t)t * n + i] = hred(e[i], P.mod[t]);
            }
            K->pk = Buf(&C, (size_t)2 * L1 * n);
            Buf ee(&C, (size_t)L1 * n), tmp(&C, (size_t)L1 * n);
            u64 *p0 = K->pk.get(), *p1 = p0 + (size_t)L1 * n;
            HIPCHK(hipMemcpyAsync(p1, a.data(), a.size() * 8, hipMemcpyHostToDevice, C.stream));
            HIPCHK(hipMemcpyAsync(ee.get(), er.data(), er.size() * 8, hipMemcpyHostToDevice, C.stream));
            ntt(C, p1, L1, 1, 0, plain_map(), false);
            ntt(C, ee.get(), L1, 1, 0, plain_map(), false);
            k_mul_pt(C.T, tmp.get(), p1, s_eval.get(), L1, 1, 0, 0, plain_map(), false, C.stream);
            k_add(C.T, p0, ee.get(), tmp.get(), L1, 1, 0, 0, 0, plain_map(), true, C.stream);
            sync(C);
        }
        // relinearisation key: s' = s^2
        {
            Buf s2(&C, sr.size());
            k_mul_pt(C.T, s2.get(), s_eval.get(), s_eval.get(), Ek, 1, 0, 0, emap, false, C.stream);
            gen_switch_key(C, *K, 0, s_eval, s2, seed);
        }
        std::vector<i64> shifts;
        for (size_t i = 0; i < nN; i++) circuit_shifts(Ns[i], what ? what : 1, shifts);
        add_rotation_keys(C, *K, shifts, seed);
        // conjugation: the real part of a Chebyshev indicator's argument
        if (nN && (what & 6)) add_galois_keys(C, *K, {(u32)(2 * C.n() - 1)}, seed);
        // base-conversion tables of every level the keys serve, so that no key
        // switch (the allocation-free rotation in particular) allocates them later
        for (int l = 0; l <= K->lmax; l++) {
            for (int j = 0; j < P.beta(l); j++) (void)modup_tab(C, l, j);
            (void)moddown_tab(C, l);
        }
        {
            std::lock_guard<std::mutex> g(g_key_seed_mu);
            g_key_seed[K.get()] = std::vector<uint8_t>(seed, seed + 32);
        }
        auto h = std::make_unique<ckr_keys>();
        h->K = std::move(K);
        *out = h.release();
    });
}

void ckr_keys_free(ckr_keys *k) {
    if (!k) return;
    {
        std::lock_guard<std::mutex> g(g_key_seed_mu);
        g_key_seed.erase(k->K.get());
    }
    delete k;
}

ckr_status ckr_keys_add_rotations(ckr_context *ctx, ckr_keys *keys, const int64_t *shifts, size_t count) {
    return guard([&] {
        NEED(ctx && keys && (shifts || !count));
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        std::vector<uint8_t> seed;
        {
            std::lock_guard<std::mutex> g(g_key_seed_mu);
            seed = g_key_seed.at(keys->K.get());
        }
        add_rotation_keys(*ctx->C, *keys->K, std::vector<i64>(shifts, shifts + count), seed.data());
    });
}

static ckr_ct *wrap(Ctx &C, DCt &&c) {
    ckr_ct *h = new ckr_ct{&C, std::move(c)};
    return h;
}

ckr_status ckr_encrypt(ckr_context *ctx, const ckr_keys *keys, const double *v, uint32_t N, uint32_t level,
                       const uint8_t seed[32], ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && v && seed && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = nullptr;
        Ctx &C = *ctx->C;
        const Keys &K = *keys->K;
        if ((int)level > K.lmax) throw Error{CKR_E_DEPTH, "level above the key level"};
        if ((u64)N > C.n() / 2) throw Error{CKR_E_RANGE, "too many slots"};
        const size_t n = C.n();
        const int L1 = (int)level + 1;
        std::vector<i64> m(n), u(n), e0(n), e1(n);
        if (!encode_slots(C.P.logn, v, N, C.P.scale[level], m.data())) throw Error{CKR_E_RANGE, "value too large"};
        {
            Stream s(seed, kEncU, 0);
            for (size_t i = 0; i < n; i++) u[i] = s.ternary();
        }
        {
            Stream s(seed, kEncE0, 0);
            for (size_t i = 0; i < n; i++) e0[i] = s.cbd21();
        }
        {
            Stream s(seed, kEncE1, 0);
            for (size_t i = 0; i < n; i++) e1[i] = s.cbd21();
        }
        // [u | e0 + m | e1] per limb
        std::vector<u64> h((size_t)3 * L1 * n);
        for (int t = 0; t < L1; t++) {
            const u64 q = C.P.mod[t];
            u64 *hu = h.data() + (size_t)t * n, *h0 = hu + (size_t)L1 * n, *h1 = h0 + (size_t)L1 * n;
            for (size_t i = 0; i < n; i++) {
                hu[i] = hred(u[i], q);
                h0[i] = hred(e0[i] + m[i], q);
                h1[i] = hred(e1[i], q);
            }
        }
        Buf dh(&C, h.size());
        HIPCHK(hipMemcpyAsync(dh.get(), h.data(), h.size() * 8, hipMemcpyHostToDevice, C.stream));
        ntt(C, dh.get(), L1, 3, (size_t)L1 * n, plain_map(), false);
        DCt c = ct_new(C, (int)level, 1);
        const size_t L = (size_t)L1 * n;
        const u64 *pk0 = K.pk.get(), *pk1 = pk0 + (size_t)(K.lmax + 1) * n;
        // c0 = u pk0 + (e0 + m), c1 = u pk1 + e1
        k_mul_pt(C.T, c.d(), pk0, dh.get(), L1, 1, 0, 0, plain_map(), false, C.stream);
        k_mul_pt(C.T, c.d() + L, pk1, dh.get(), L1, 1, 0, 0, plain_map(), false, C.stream);
        k_add(C.T, c.d(), c.d(), dh.get() + L, L1, 2, L, L, L, plain_map(), false, C.stream);
        sync(C);
        *out = wrap(C, std::move(c));
    });
}

// coefficient-domain copy of a ciphertext, downloaded
static std::vector<u64> download_coeffs(Ctx &C, const DCt &c) {
    DCt t = ev_copy(C, c);
    const size_t L = (size_t)(c.level + 1) * C.n();
    ntt(C, t.d(), c.level + 1, 2 * c.B, L, plain_map(), true);
    std::vector<u64> h((size_t)c.B * 2 * L);
    HIPCHK(hipMemcpyAsync(h.data(), t.d(), h.size() * 8, hipMemcpyDeviceToHost, C.stream));
    sync(C);
    return h;
}

ckr_status ckr_decrypt(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *ct, double *out, uint32_t count) {
    return guard([&] {
        NEED(ctx && keys && ct && (out || !count));
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        const Keys &K = *keys->K;
        const size_t n = C.n();
        if ((u64)count > n / 2) throw Error{CKR_E_RANGE, "too many slots"};
        // c0 + c1 s on q_0 (valid while |m| < q_0 / 2); s uploaded only for this call
        const u64 q = C.P.mod[0];
        std::vector<u64> s0(n);
        for (size_t i = 0; i < n; i++) s0[i] = hred(K.s[i], q);
        Buf ds(&C, n), x(&C, n);
        HIPCHK(hipMemcpyAsync(ds.get(), s0.data(), n * 8, hipMemcpyHostToDevice, C.stream));
        ntt(C, ds.get(), 1, 1, 0, plain_map(), false);
        const u64 *c0 = ct->ct.d(), *c1 = c0 + (size_t)(ct->ct.level + 1) * n;
        k_mul_pt(C.T, x.get(), c1, ds.get(), 1, 1, 0, 0, plain_map(), false, C.stream);
        k_add(C.T, x.get(), x.get(), c0, 1, 1, 0, 0, 0, plain_map(), false, C.stream);
        ntt(C, x.get(), 1, 1, 0, plain_map(), true);
        std::vector<u64> h(n);
        HIPCHK(hipMemcpyAsync(h.data(), x.get(), n * 8, hipMemcpyDeviceToHost, C.stream));
        sync(C);
        std::vector<i64> m(n);
        for (size_t i = 0; i < n; i++) m[i] = h[i] > q / 2 ? -(i64)(q - h[i]) : (i64)h[i];
        decode_slots(C.P.logn, m.data(), C.P.scale[ct->ct.level], count, out);
    });
}

uint32_t ckr_ct_level(const ckr_ct *ct) { return ct ? (uint32_t)ct->ct.level : 0; }
double ckr_ct_scale(const ckr_ct *ct) { return ct ? ct->C->P.scale[ct->ct.level] : 0.0; }
void ckr_ct_free(ckr_ct *ct) { delete ct; }

ckr_status ckr_ct_export(ckr_context *ctx, const ckr_ct *ct, uint64_t *data, size_t words) {
    return guard([&] {
        NEED(ctx && ct && data);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        const size_t need = (size_t)2 * (ct->ct.level + 1) * C.n();
        if (words < need) throw Error{CKR_E_INVALID, "export buffer too small"};
        std::vector<u64> h = download_coeffs(C, ct->ct);
        std::memcpy(data, h.data(), need * 8);
    });
}

ckr_status ckr_ct_import(ckr_context *ctx, const uint64_t *data, size_t words, uint32_t level, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && data && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = nullptr;
        Ctx &C = *ctx->C;
        if ((int)level > C.P.L) throw Error{CKR_E_DEPTH, "level above the chain"};
        const size_t L = (size_t)(level + 1) * C.n();
        if (words != 2 * L) throw Error{CKR_E_INVALID, "word count does not match level"};
        for (int p = 0; p < 2; p++)
            for (u32 t = 0; t <= level; t++) {
                const u64 q = C.P.mod[t];
                const uint64_t *x = data + p * L + (size_t)t * C.n();
                for (size_t i = 0; i < C.n(); i++)
                    if (x[i] >= q) throw Error{CKR_E_INVALID, "residue not below its modulus"};
            }
        DCt c = ct_new(C, (int)level, 1);
        HIPCHK(hipMemcpyAsync(c.d(), data, 2 * L * 8, hipMemcpyHostToDevice, C.stream));
        ntt(C, c.d(), (int)level + 1, 2, L, plain_map(), false);
        sync(C);
        *out = wrap(C, std::move(c));
    });
}

uint32_t ckr_rank_depth(ckr_sign cmp, int tie) { return rank_depth(cmp, tie); }
uint32_t ckr_argmin_depth(ckr_sign cmp, ckr_sign ind) { return argmin_depth(cmp, ind); }
uint32_t ckr_rank_multi_depth(ckr_sign cmp) { return rank_multi_depth(cmp); }
uint32_t ckr_sort_multi_depth(ckr_sign cmp, ckr_sign ind) { return sort_multi_depth(cmp, ind); }
uint32_t ckr_order_stat_depth(uint32_t N, uint32_t k, ckr_sign cmp, ckr_sign ind, int tie_correct) {
    return order_stat_depth((int)N, (int)k, cmp, ind, tie_correct != 0);
}
uint32_t ckr_sort_depth(ckr_sign cmp, ckr_sign ind) { return sort_depth(cmp, ind); }
uint32_t ckr_sort_col_depth(ckr_sign cmp, ckr_sign ind) { return sort_col_depth(cmp, ind); }
uint32_t ckr_rank_depth_n(uint32_t N, ckr_sign cmp, int tie) { return rank_depth_n((int)N, cmp, tie); }

ckr_status ckr_rank(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *v, uint32_t N, ckr_sign cmp, int tie,
                    ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && v && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = nullptr;
        Ctx &C = *ctx->C;
        DCt r = tie ? tie_rank(C, *keys->K, v->ct, (int)N, cmp) : rank(C, *keys->K, v->ct, (int)N, cmp);
        *out = wrap(C, std::move(r));
    });
}

// outputs of batch entry i: out[i] (rank, sort) or out[2i], out[2i+1] (argmin one-hot, value)
ckr_status ckr_run_batch(ckr_context *ctx, const ckr_keys *keys, int kind, uint32_t N, ckr_sign cmp, ckr_sign ind,
                         const ckr_ct *const *v, size_t count, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && v && out && count);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        std::vector<const DCt *> in;
        for (size_t i = 0; i < count; i++) {
            NEED(v[i]);
            in.push_back(&v[i]->ct);
        }
        std::vector<DCt> outs = run_kind(C, *keys->K, kind, (int)N, cmp, ind, in);
        const size_t per = outs.size();
        std::vector<ckr_ct *> made;
        for (size_t i = 0; i < count; i++)
            for (size_t k = 0; k < per; k++) made.push_back(wrap(C, slice(C, outs[k], (int)i, 1)));
        for (size_t i = 0; i < made.size(); i++) out[i] = made[i];
    });
}

ckr_status ckr_rank_batch(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *const *v, size_t count, uint32_t N,
                          ckr_sign cmp, ckr_ct **out) {
    return ckr_run_batch(ctx, keys, kRankCircuit, N, cmp, ckr_sign{0, 0}, v, count, out);
}

struct ckr_server {
    std::unique_ptr<Server> S;
};

ckr_status ckr_server_create(size_t hbm_budget, uint32_t max_batch, ckr_server **out) {
    return guard([&] {
        NEED(out);
        auto h = std::make_unique<ckr_server>();
        h->S = std::make_unique<Server>(hbm_budget, (int)max_batch);
        *out = h.release();
    });
}

ckr_status ckr_server_add_route(ckr_server *srv, int kind, uint32_t N, ckr_context *ctx, const ckr_keys *keys,
                                ckr_sign cmp, ckr_sign ind) {
    return guard([&] {
        NEED(srv && ctx && keys);
        if (kind < 1 || kind > 3) throw Error{CKR_E_INVALID, "kind"};
        if (kind == kRankCircuit) check_N_padded(*ctx->C, N);
        else check_N(*ctx->C, N);
        Route r{kind, (int)N, ctx->C.get(), keys->K.get(), cmp, ind};
        srv->S->add_route(r);
    });
}

ckr_status ckr_server_submit(ckr_server *srv, int kind, uint32_t N, const ckr_ct *v, uint64_t *ticket) {
    return guard([&] {
        NEED(srv && v && ticket);
        *ticket = srv->S->submit(kind, (int)N, v->ct);
    });
}

ckr_status ckr_server_wait(ckr_server *srv, uint64_t ticket, int timeout_ms, ckr_ct **outs, size_t n_outs,
                           double *latency_ms) {
    std::vector<DCt> o;
    std::string err;
    int st = CKR_OK;
    Ctx *C = nullptr;
    ckr_status g = guard([&] {
        NEED(srv && (outs || !n_outs));
        st = srv->S->wait(ticket, timeout_ms, o, latency_ms, err, &C);
    });
    if (g != CKR_OK) return g;
    if (st != CKR_OK) {
        g_last_error = err.empty() ? "request failed" : err;
        return (ckr_status)st;
    }
    if (o.size() > n_outs) {
        g_last_error = "output array too small";
        return CKR_E_INVALID;
    }
    for (size_t i = 0; i < o.size(); i++) outs[i] = new ckr_ct{C, std::move(o[i])};
    return CKR_OK;
}

ckr_status ckr_server_stats(ckr_server *srv, double *stats) {
    return guard([&] {
        NEED(srv && stats);
        srv->S->stats(stats);
    });
}

void ckr_server_free(ckr_server *srv) { delete srv; }

ckr_status ckr_context_set_graphs(ckr_context *ctx, int enable) {
    return guard([&] {
        NEED(ctx);
        ctx->C->graphs = enable != 0;
    });
}

ckr_status ckr_argmin(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *v, uint32_t N, ckr_sign cmp,
                      ckr_sign ind, ckr_ct **onehot, ckr_ct **value) {
    return guard([&] {
        NEED(ctx && keys && v && onehot && value);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *onehot = *value = nullptr;
        Ctx &C = *ctx->C;
        DCt oh, val;
        order_stat(C, *keys->K, v->ct, (int)N, 1, 1, cmp, ind, oh, val);
        *onehot = wrap(C, std::move(oh));
        *value = wrap(C, std::move(val));
    });
}

ckr_status ckr_order_stat(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *v, uint32_t N, uint32_t k,
                          ckr_sign cmp, ckr_sign ind, int tie_correct, ckr_ct **onehot, ckr_ct **value) {
    return guard([&] {
        NEED(ctx && keys && v && onehot && value);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *onehot = *value = nullptr;
        Ctx &C = *ctx->C;
        DCt oh, val;
        order_stat(C, *keys->K, v->ct, (int)N, (int)k, tie_correct != 0, cmp, ind, oh, val);
        *onehot = wrap(C, std::move(oh));
        *value = wrap(C, std::move(val));
    });
}

uint32_t ckr_order_range_depth(uint32_t N, uint32_t a, uint32_t b, ckr_sign cmp, ckr_sign ind, int tie_correct) {
    return order_range_depth((int)N, (int)a, (int)b, cmp, ind, tie_correct != 0);
}

ckr_status ckr_order_range(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *const *v, size_t count, uint32_t N,
                           uint32_t a, uint32_t b, ckr_sign cmp, ckr_sign ind, int tie_correct, ckr_ct **onehot,
                           ckr_ct **value) {
    return guard([&] {
        NEED(ctx && keys && v && count && onehot && value);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        check_N_padded(C, N);
        // every argument error before the first launch
        if (a < 1 || a > b || b > N) throw Error{CKR_E_INVALID, "the rank window must satisfy 1 <= a <= b <= N"};
        if (a == 1 && b == N) throw Error{CKR_E_INVALID, "the rank window [1, N] selects every element"};
        if (pow2_ceil((int)N) != (int)N && !tie_correct)
            throw Error{CKR_E_INVALID, "N that is not a power of two needs tie-correction"};
        if (!sign_valid(cmp) || !sign_valid(ind)) throw Error{CKR_E_INVALID, "empty comparator"};
        Spec s;
        s.kind = kOrderCircuit;
        s.N = (int)N;
        s.k = (int)a;
        s.k_hi = (int)b;
        s.tie = tie_correct != 0;
        s.cmp = cmp;
        s.ind = ind;
        std::vector<const DCt *> in;
        for (size_t i = 0; i < count; i++) {
            NEED(v[i]);
            in.push_back(&v[i]->ct);
        }
        std::vector<std::vector<DCt>> r = run_groups(C, *keys->K, {s}, {in});
        std::vector<ckr_ct *> made;
        for (size_t i = 0; i < count; i++) {
            made.push_back(wrap(C, slice(C, r[0][0], (int)i, 1)));
            made.push_back(wrap(C, slice(C, r[0][1], (int)i, 1)));
        }
        for (size_t i = 0; i < count; i++) {
            onehot[i] = made[2 * i];
            value[i] = made[2 * i + 1];
        }
    });
}

ckr_status ckr_rank_multi(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *const *blocks, uint32_t L, uint32_t b,
                          ckr_sign cmp, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && blocks && out && L);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        std::vector<const DCt *> in;
        for (u32 i = 0; i < L; i++) {
            NEED(blocks[i]);
            if (blocks[i]->ct.B != 1 || blocks[i]->ct.level != blocks[0]->ct.level)
                throw Error{CKR_E_INVALID, "blocks must be single ciphertexts of one level"};
            in.push_back(&blocks[i]->ct);
        }
        DCt R = rank_multi(C, *keys->K, stack(C, in), (int)b, cmp);
        std::vector<ckr_ct *> made;
        for (u32 i = 0; i < L; i++) made.push_back(wrap(C, slice(C, R, (int)i, 1)));
        for (u32 i = 0; i < L; i++) out[i] = made[i];
    });
}

ckr_status ckr_sort_multi(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *const *blocks, uint32_t L, uint32_t b,
                          ckr_sign cmp, ckr_sign ind, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && blocks && out && L);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        std::vector<const DCt *> in;
        for (u32 i = 0; i < L; i++) {
            NEED(blocks[i]);
            if (blocks[i]->ct.B != 1 || blocks[i]->ct.level != blocks[0]->ct.level)
                throw Error{CKR_E_INVALID, "blocks must be single ciphertexts of one level"};
            in.push_back(&blocks[i]->ct);
        }
        DCt S = sort_multi(C, *keys->K, stack(C, in), (int)b, cmp, ind);
        std::vector<ckr_ct *> made;
        for (u32 i = 0; i < L; i++) made.push_back(wrap(C, slice(C, S, (int)i, 1)));
        for (u32 i = 0; i < L; i++) out[i] = made[i];
    });
}

ckr_status ckr_run_mixed(ckr_context *ctx, const ckr_keys *keys, const ckr_query *q, size_t count, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && q && out && count);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        // group queries by (circuit, level) in order of first appearance
        std::vector<Spec> specs;
        std::vector<int> levels;
        std::vector<std::vector<const DCt *>> in;
        std::vector<std::pair<int, int>> where(count);  // (group, index in group)
        for (size_t i = 0; i < count; i++) {
            NEED(q[i].v);
            const Spec s = spec_of(C, q[i].kind, (int)q[i].N, (int)q[i].k, q[i].tie_correct, q[i].cmp, q[i].ind);
            const int level = q[i].v->ct.level;
            int g = 0;
            while (g < (int)specs.size() && !(specs[g].tup() == s.tup() && levels[g] == level)) g++;
            if (g == (int)specs.size()) {
                specs.push_back(s);
                levels.push_back(level);
                in.emplace_back();
            }
            where[i] = {g, (int)in[g].size()};
            in[g].push_back(&q[i].v->ct);
        }
        std::vector<std::vector<DCt>> outs = run_groups(C, *keys->K, specs, in);
        std::vector<ckr_ct *> made(2 * count, nullptr);
        for (size_t i = 0; i < count; i++) {
            const auto [g, j] = where[i];
            for (size_t o = 0; o < outs[g].size(); o++) made[2 * i + o] = wrap(C, slice(C, outs[g][o], j, 1));
        }
        for (size_t i = 0; i < made.size(); i++) out[i] = made[i];
    });
}

ckr_status ckr_sort(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *v, uint32_t N, ckr_sign cmp, ckr_sign ind,
                    ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && v && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = nullptr;
        Ctx &C = *ctx->C;
        DCt r = sort(C, *keys->K, v->ct, (int)N, cmp, ind);
        *out = wrap(C, std::move(r));
    });
}

uint32_t ckr_order_stat_div_depth(uint32_t N, uint32_t k, ckr_sign cmp, ckr_sign ind, uint32_t iters) {
    return order_stat_div_depth((int)N, (int)k, cmp, ind, (int)iters);
}

ckr_status ckr_order_stat_div(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *const *v, size_t count, uint32_t N,
                              uint32_t k, ckr_sign cmp, ckr_sign ind, uint32_t iters, ckr_ct **onehot,
                              ckr_ct **value) {
    return guard([&] {
        NEED(ctx && keys && v && count && onehot && value);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        std::vector<const DCt *> in;
        for (size_t i = 0; i < count; i++) {
            NEED(v[i]);
            if (v[i]->ct.level != v[0]->ct.level) throw Error{CKR_E_INVALID, "inputs at different levels"};
            in.push_back(&v[i]->ct);
        }
        DCt X, oh, val;
        const DCt *xp = &v[0]->ct;
        if (count > 1) {
            X = stack(C, in);
            xp = &X;
        }
        order_stat_div(C, *keys->K, *xp, (int)N, (int)k, cmp, ind, (int)iters, oh, val);
        for (size_t i = 0; i < count; i++) {
            onehot[i] = wrap(C, slice(C, oh, (int)i, 1));
            value[i] = wrap(C, slice(C, val, (int)i, 1));
        }
    });
}

ckr_status ckr_sort_col(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *v, uint32_t N, ckr_sign cmp,
                        ckr_sign ind, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && v && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = nullptr;
        Ctx &C = *ctx->C;
        DCt r = sort_col(C, *keys->K, v->ct, (int)N, cmp, ind);
        *out = wrap(C, std::move(r));
    });
}

ckr_status ckr_op_rotate(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *a, int64_t k, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && a && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = wrap(*ctx->C, ev_rotate(*ctx->C, *keys->K, a->ct, k));
    });
}
ckr_status ckr_op_rotate_into(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *a, int64_t k, ckr_ct *out) {
    return guard([&] {
        NEED(ctx && keys && a && out);
        Ctx &C = *ctx->C;
        std::lock_guard<std::recursive_mutex> lk_(C.mu_run);
        const DCt &x = a->ct;
        const DCt &y = out->ct;
        if (a->C != &C || out->C != &C || keys->K->C != &C) throw Error{CKR_E_INVALID, "handles of another context"};
        if (x.B != 1 || y.B != 1 || x.level != y.level)
            throw Error{CKR_E_INVALID, "out must be a single ciphertext at the input's level"};
        if (x.d() == y.d()) throw Error{CKR_E_INVALID, "out must not be the input"};
        const int l = x.level;
        if (l > keys->K->lmax) throw Error{CKR_E_DEPTH, "ciphertext above key level"};
        const size_t n = C.n(), L = (size_t)(l + 1) * n;
        const u32 g = galois_left(C, k);
        if (g == 1) {  // a rotation by a multiple of n/2 slots: the identity
            HIPCHK(hipMemcpyAsync(y.d(), x.d(), 2 * L * 8, hipMemcpyDeviceToDevice, C.stream));
            return;
        }
        const size_t need = keyswitch_scratch_words(C, l);
        if (need > kScratchWords)
            throw Error{CKR_E_NOMEM, "the allocation-free rotation needs " + std::to_string(need * 8 >> 20) +
                                         " MiB of scratch at this ring and level; it has " +
                                         std::to_string(kScratchWords * 8 >> 20) + " MiB"};
        const Buf &key = find_key(*keys->K, g);
        {
            std::lock_guard<std::mutex> tg(C.mu);
            bool have = C.moddown.count(l) != 0;
            for (int j = 0; j < C.P.beta(l); j++) have = have && C.modup.count(std::make_pair(l, j));
            if (!have) throw Error{CKR_E_INVALID, "base-conversion tables of this level are missing"};
        }
        if (!C.scratch) throw Error{CKR_E_DEVICE, "scratch array unavailable"};
        struct Arena {
            Pool &p;
            ~Arena() { p.clear_arena(); }
        } arena{C.pool};
        C.pool.set_arena(C.scratch, kScratchWords * 8);
        keyswitch(C, *keys->K, key, x.d() + L, 2 * L, l, 1, y.d(), 2 * L, L, x.d(), 2 * L, L, 1, nullptr, 0, 0, 0,
                  g);
    });
}
ckr_status ckr_op_mul(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *a, const ckr_ct *b, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && a && b && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = wrap(*ctx->C, ev_mul(*ctx->C, *keys->K, a->ct, b->ct));
    });
}
ckr_status ckr_op_cheb_eval(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *a, const double *coeffs,
                            uint32_t deg1, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && a && coeffs && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = wrap(*ctx->C, cheb_eval(*ctx->C, *keys->K, a->ct, std::vector<double>(coeffs, coeffs + deg1)));
    });
}
ckr_status ckr_op_cmp_sign(ckr_context *ctx, const ckr_keys *keys, const ckr_ct *a, ckr_sign cmp, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && keys && a && out);
        check_sign(cmp);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = wrap(*ctx->C, cmp_sign(*ctx->C, *keys->K, a->ct, cmp));
    });
}
ckr_status ckr_op_add(ckr_context *ctx, const ckr_ct *a, const ckr_ct *b, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && a && b && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = wrap(*ctx->C, ev_add(*ctx->C, a->ct, b->ct, false));
    });
}
ckr_status ckr_op_sub(ckr_context *ctx, const ckr_ct *a, const ckr_ct *b, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && a && b && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = wrap(*ctx->C, ev_add(*ctx->C, a->ct, b->ct, true));
    });
}
ckr_status ckr_op_rescale(ckr_context *ctx, const ckr_ct *a, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && a && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = wrap(*ctx->C, ev_rescale(*ctx->C, a->ct));
    });
}
ckr_status ckr_op_cmul_to(ckr_context *ctx, const ckr_ct *a, double c, uint32_t target, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && a && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = wrap(*ctx->C, ev_cmul_to(*ctx->C, a->ct, c, (int)target));
    });
}
ckr_status ckr_op_add_const(ckr_context *ctx, const ckr_ct *a, double c, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && a && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        *out = wrap(*ctx->C, ev_add_const(*ctx->C, a->ct, c));
    });
}
ckr_status ckr_op_mul_plain(ckr_context *ctx, const ckr_ct *a, const double *z, uint32_t count, ckr_ct **out) {
    return guard([&] {
        NEED(ctx && a && z && out);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        if ((u64)count > C.n() / 2) throw Error{CKR_E_RANGE, "too many slots"};
        Buf pt = encode_plain(C, std::vector<double>(z, z + count), a->ct.level);
        *out = wrap(C, ev_mul_plain(C, a->ct, pt));
    });
}

ckr_status ckr_ntt_device(ckr_context *ctx, uint64_t *data, uint32_t limbs, uint32_t first_mod, int inverse) {
    return guard([&] {
        NEED(ctx && data);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        if (first_mod + limbs > (u32)C.P.nmod()) throw Error{CKR_E_INVALID, "modulus index out of range"};
        ntt(C, data, (int)limbs, 1, 0, plain_map((int)first_mod), inverse != 0);
        HIPCHK(hipGetLastError());
    });
}

ckr_status ckr_set_profiling(ckr_context *ctx, int enable) {
    return guard([&] {
        NEED(ctx);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        prof_resolve(C);
        C.prof.on = enable != 0;
    });
}

ckr_status ckr_profile_reset(ckr_context *ctx) {
    return guard([&] {
        NEED(ctx);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        prof_resolve(C);
        for (int c = 0; c < kNCat; c++) C.prof.launches[c] = 0, C.prof.ms[c] = 0, C.prof.bytes[c] = 0;
    });
}

ckr_status ckr_profile_read(ckr_context *ctx, int category, uint64_t *launches, double *total_ms, double *bytes) {
    return guard([&] {
        NEED(ctx);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        if (category < 0 || category >= kNCat) throw Error{CKR_E_INVALID, "profile category"};
        Ctx &C = *ctx->C;
        prof_resolve(C);
        if (launches) *launches = C.prof.launches[category];
        if (total_ms) *total_ms = C.prof.ms[category];
        if (bytes) *bytes = C.prof.bytes[category];
    });
}

const char *ckr_profile_name(int category) { return category >= 0 && category < kNCat ? kCatName[category] : nullptr; }

// Time every NTT tile variant on `limbs` limbs of zeros (timing does not depend
// on the values) and keep the fastest per (direction, pass).  ms receives
// [inverse][pass][variant] averages (2*2*kNttVariants floats) when not NULL.
ckr_status ckr_autotune(ckr_context *ctx, uint32_t limbs, uint32_t iters, float *ms) {
    return guard([&] {
        NEED(ctx);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        if (limbs == 0 || limbs > (u32)C.P.nmod() * 64) throw Error{CKR_E_INVALID, "limbs"};
        iters = std::max(1u, iters);
        const size_t n = C.n();
        Buf buf(&C, (size_t)limbs * n);
        HIPCHK(hipMemsetAsync(buf.get(), 0, (size_t)limbs * n * 8, C.stream));
        // limbs cycle through the q chain
        const int nq = C.P.nq;
        std::vector<hipEvent_t> ev(2);
        for (auto &e : ev) HIPCHK(hipEventCreate(&e));
        for (int inv = 0; inv < 2; inv++)
            for (int pass = 0; pass < 2; pass++) {
                float best = 1e30f;
                int bestv = 0;
                for (int v = 0; v < kNttVariants; v++) {
                    // one launch over whole polynomials of nq limbs (the shape the circuits
                    // issue), then the remainder
                    auto launch = [&] {
                        const u32 full = limbs / (u32)nq, rest = limbs - full * (u32)nq;
                        if (full) {
                            LimbBatch b{buf.get(), nq, (int)full, (size_t)nq * n, plain_map()};
                            k_ntt_pass_variant(C.T, b, inv != 0, pass, v, C.stream);
                        }
                        if (rest) {
                            LimbBatch b{buf.get() + (size_t)full * nq * n, (int)rest, 1, 0, plain_map()};
                            k_ntt_pass_variant(C.T, b, inv != 0, pass, v, C.stream);
                        }
                    };
                    launch();  // warm
                    HIPCHK(hipEventRecord(ev[0], C.stream));
                    for (u32 it = 0; it < iters; it++) launch();
                    HIPCHK(hipEventRecord(ev[1], C.stream));
                    HIPCHK(hipEventSynchronize(ev[1]));
                    float t = 0;
                    HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
                    t /= (float)iters;
                    if (ms) ms[(inv * 2 + pass) * kNttVariants + v] = t;
                    if (t < best) best = t, bestv = v;
                }
                C.T.ntt_variant[inv][pass] = bestv;
            }
        C.tune_epoch++;
        for (auto &e : ev) (void)hipEventDestroy(e);
    });
}

ckr_status ckr_autotune_row_ip(ckr_context *ctx, uint32_t batch, uint32_t iters, float *ms) {
    return guard([&] {
        NEED(ctx);
        if (batch == 0 || batch > 4096) throw Error{CKR_E_INVALID, "batch"};
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        Ctx &C = *ctx->C;
        const Params &P = C.P;
        iters = std::max(1u, iters);
        const size_t n = C.n();
        const int l = P.nq - 1, E = l + 1 + P.K, beta = P.beta(l);
        const int B = (int)batch;
        Buf d(&C, (size_t)B * (l + 1) * n), ext(&C, (size_t)B * beta * E * n), key(&C, (size_t)beta * 2 * E * n),
            acc(&C, (size_t)B * 2 * E * n);
        for (const Buf *b : {&d, &ext, &key})
            HIPCHK(hipMemsetAsync(b->get(), 0, b->words() * 8, C.stream));
        IPArgs ia;
        ia.d = d.get();
        ia.ext = ext.get();
        ia.key = key.get();
        ia.accb = acc.get();
        ia.acca = acc.get() + (size_t)E * n;
        ia.level = l;
        ia.E = E;
        ia.beta = beta;
        ia.alpha = P.alpha;
        ia.Ek = E;
        ia.lmax_key = l;
        ia.nq = P.nq;
        ia.B = B;
        ia.sd = (size_t)(l + 1) * n;
        ia.sext = (size_t)beta * E * n;
        ia.sacc = (size_t)2 * E * n;
        ia.inv_p = true;  // as in the key switch
        hipEvent_t ev[2];
        for (auto &e : ev) HIPCHK(hipEventCreate(&e));
        const int keep = C.T.row_ip_variant;
        float best = 1e30f;
        int bestv = keep;
        for (int v = 0; v < kRowIpVariants; v++) {
            C.T.row_ip_variant = v;
            k_ntt_row_ip(C.T, ia, C.stream);  // warm
            HIPCHK(hipEventRecord(ev[0], C.stream));
            for (u32 it = 0; it < iters; it++) k_ntt_row_ip(C.T, ia, C.stream);
            HIPCHK(hipEventRecord(ev[1], C.stream));
            HIPCHK(hipEventSynchronize(ev[1]));
            float t = 0;
            HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
            t /= (float)iters;
            if (ms) ms[v] = t;
            if (t < best) best = t, bestv = v;
        }
        C.T.row_ip_variant = bestv;
        C.tune_epoch++;
        for (auto &e : ev) (void)hipEventDestroy(e);
    });
}

ckr_status ckr_set_ntt_chunk(ckr_context *ctx, uint32_t limbs) {
    return guard([&] {
        NEED(ctx);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        ctx->C->ntt_chunk = (int)limbs;
        ctx->C->tune_epoch++;
    });
}

ckr_status ckr_ntt_variant(ckr_context *ctx, int inverse, int pass, int variant) {
    return guard([&] {
        NEED(ctx);
        if (inverse < 0 || inverse > 1 || pass < 0 || pass > 1 || variant < 0 || variant >= kNttVariants)
            throw Error{CKR_E_INVALID, "variant"};
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        ctx->C->T.ntt_variant[inverse][pass] = variant;
        ctx->C->tune_epoch++;
    });
}

ckr_status ckr_row_ip_variant(ckr_context *ctx, int variant) {
    return guard([&] {
        NEED(ctx);
        if (variant < 0 || variant >= kRowIpVariants) throw Error{CKR_E_INVALID, "variant"};
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        ctx->C->T.row_ip_variant = variant;
        ctx->C->tune_epoch++;
    });
}

ckr_status ckr_synchronize(ckr_context *ctx) {
    return guard([&] {
        NEED(ctx);
        std::lock_guard<std::recursive_mutex> lk_(ctx->C->mu_run);
        sync(*ctx->C);
    });
}

}  // extern "C"
