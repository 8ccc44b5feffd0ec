// Derivation of the B_nl / C_nl gather tables; see asp_tables.hpp for the
// mathematics and the paper passages it follows.
#include "asp_tables.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <atomic>
#include <exception>
#include <new>
#include <thread>
#include <stdexcept>
#include <string>
#include <unordered_map>

namespace fcc {

const std::vector<std::array<int, 9>>& weyl_group() {
  static const std::vector<std::array<int, 9>> G = [] {
    const int gen[3][9] = {{-1, 0, 0, 1, 1, 0, 0, 0, 1},
                           {1, 1, 0, 0, -1, 0, 0, 1, 1},
                           {1, 0, 0, 0, 1, 1, 0, 0, -1}};
    std::vector<std::array<int, 9>> out{{1, 0, 0, 0, 1, 0, 0, 0, 1}};
    for (size_t h = 0; h < out.size(); ++h)
      for (const auto& s : gen) {
        std::array<int, 9> p{};
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) p[3 * i + j] += s[3 * i + k] * out[h][3 * k + j];
        if (std::find(out.begin(), out.end(), p) == out.end()) out.push_back(p);
      }
    if (out.size() != 24) throw std::logic_error("Weyl group closure");
    return out;
  }();
  return G;
}

void dominant(int& a, int& b, int& c) {
  for (;;) {
    if (a < 0) {        // s1: (a,b,c) -> (-a, a+b, c)
      b += a;
      a = -a;
    } else if (b < 0) { // s2: (a,b,c) -> (a+b, -b, b+c)
      a += b;
      c += b;
      b = -b;
    } else if (c < 0) { // s3: (a,b,c) -> (a, b+c, -c)
      b += c;
      c = -c;
    } else {
      return;
    }
  }
}

namespace {

constexpr int K = 8;  // monomial slots per polynomial
using Coef = std::array<double, K>;

struct QKey {
  long long q[K];
  bool operator==(const QKey& o) const { return std::memcmp(q, o.q, sizeof q) == 0; }
};
struct QHash {
  size_t operator()(const QKey& k) const {
    uint64_t h = 1469598103934665603ull;
    for (long long v : k.q) h = (h ^ uint64_t(v)) * 1099511628211ull;
    return size_t(h ^ (h >> 29));
  }
};
QKey quantise(const Coef& p) {
  QKey key;
  for (int i = 0; i < K; ++i) key.q[i] = std::llround(p[i] * 1073741824.0);  // 2^30
  return key;
}

// Polynomial pool shared by all threads: append-only storage with a fixed
// capacity (readers index it without locks), a locked index for interning,
// and per-thread caches in front of it.
struct PolyPool {
  static constexpr uint32_t kCap = 1u << 16;
  std::vector<Coef> polys;
  std::atomic<uint32_t> count{0};
  std::atomic<int> slot_of_code[64];
  int code_of_slot[K];
  std::atomic<int> nslots{0};
  std::mutex mu;
  std::unordered_map<QKey, uint32_t, QHash> index;
  uint64_t generation;
  PolyPool() : polys(kCap) {
    static std::atomic<uint64_t> gen{1};
    generation = gen++;
    for (auto& s : slot_of_code) s.store(-1);
    slot(0);  // the constant monomial is slot 0
  }
  int slot(int code) {
    int s = slot_of_code[code].load(std::memory_order_acquire);
    if (s >= 0) return s;
    std::lock_guard<std::mutex> lock(mu);
    s = slot_of_code[code].load();
    if (s >= 0) return s;
    s = nslots.load();
    if (s >= K) throw std::runtime_error("too many monomials");
    code_of_slot[s] = code;
    nslots.store(s + 1, std::memory_order_release);
    slot_of_code[code].store(s, std::memory_order_release);
    return s;
  }
  const Coef& at(uint32_t id) const { return polys[id]; }
  // The exact coefficients are rationals whose denominators divide 144 (the
  // orbit weights 1/24, 1/|O| of the product and reduction formulas); the
  // computed ones carry rounding that depends on the order in which threads
  // derived them.  Snapping to k/144 makes every interned value, and so the
  // tables, independent of thread timing.  Values that are not that close to
  // such a rational are kept as computed.
  static Coef snap(Coef p) {
    for (double& v : p) {
      const double q = std::nearbyint(v * 144.0);
      if (std::fabs(v * 144.0 - q) < 1e-7) v = q / 144.0;
    }
    return p;
  }
  uint32_t intern(const Coef& raw) {
    const Coef p = snap(raw);
    thread_local uint64_t cache_gen = 0;
    thread_local std::unordered_map<QKey, uint32_t, QHash> cache;
    if (cache_gen != generation) {
      cache.clear();
      cache_gen = generation;
    }
    QKey key = quantise(p);
    auto c = cache.find(key);
    if (c != cache.end()) return c->second;
    uint32_t id;
    {
      std::lock_guard<std::mutex> lock(mu);
      auto it = index.find(key);
      if (it != index.end()) {
        id = it->second;
      } else {
        id = count.load();
        if (id >= kCap) throw std::runtime_error("too many polynomials");
        polys[id] = p;
        index.emplace(key, id);
        count.store(id + 1, std::memory_order_release);
      }
    }
    cache.emplace(key, id);
    return id;
  }
  // exponent-wise sum of two monomial codes (base-4 digits), -1 on overflow
  static int add_codes(int a, int b) {
    int out = 0, mul = 1;
    for (int d = 0; d < 3; ++d) {
      int e = (a % 4) + (b % 4);
      if (e > 3) return -1;
      out += e * mul;
      a /= 4;
      b /= 4;
      mul *= 4;
    }
    return out;
  }
};

using SVec = std::vector<std::pair<uint32_t, uint32_t>>;  // (key, poly id)

// Dense accumulator over a few keys.
struct Acc {
  std::vector<uint32_t> keys;
  std::vector<Coef> vals;
  void clear() {
    keys.clear();
    vals.clear();
  }
  Coef& at(uint32_t key) {
    for (size_t i = 0; i < keys.size(); ++i)
      if (keys[i] == key) return vals[i];
    keys.push_back(key);
    vals.push_back(Coef{});
    return vals.back();
  }
  SVec finish(PolyPool& pool) {
    SVec out;
    out.reserve(keys.size());
    for (size_t i = 0; i < keys.size(); ++i) {
      Coef c = vals[i];
      double mx = 0.0;
      for (double v : c) mx = std::max(mx, std::fabs(v));
      if (mx < 1e-11) continue;
      for (double& v : c)
        if (std::fabs(v) < 1e-11) v = 0.0;
      out.emplace_back(keys[i], pool.intern(c));
    }
    std::sort(out.begin(), out.end());
    return out;
  }
};

// Reduction of indices modulo the skew ideal and product expansions of C
// columns.  One instance per thread (its memo is private); the pool is shared.
struct Deriver {
  int nl, m;
  PolyPool& pool;
  std::array<std::vector<std::array<int, 3>>, 3> orbit_e;   // distinct W e_d
  std::array<std::vector<std::array<int, 3>>, 8> orbit_def; // g def for all 24 g
  std::unordered_map<uint64_t, SVec> red_memo;             // out-of-range indices only
  uint32_t one_pid;

  Deriver(int nl_, PolyPool& pool_) : nl(nl_), m(nl_ / 2), pool(pool_) {
    const auto& G = weyl_group();
    for (int d = 0; d < 3; ++d) {
      for (const auto& g : G) {
        std::array<int, 3> v{g[d], g[3 + d], g[6 + d]};  // g e_d = column d
        if (std::find(orbit_e[d].begin(), orbit_e[d].end(), v) == orbit_e[d].end())
          orbit_e[d].push_back(v);
      }
    }
    for (int f = 0; f < 8; ++f) {
      int de[3] = {(f >> 2) & 1, (f >> 1) & 1, f & 1};
      for (const auto& g : G) {
        std::array<int, 3> v;
        for (int i = 0; i < 3; ++i) v[i] = g[3 * i] * de[0] + g[3 * i + 1] * de[1] + g[3 * i + 2] * de[2];
        orbit_def[f].push_back(v);
      }
    }
    Coef one{};
    one[0] = 1.0;
    one_pid = pool.intern(one);
  }
  static uint64_t key3(int a, int b, int c) {
    return (uint64_t(uint32_t(a)) << 42) | (uint64_t(uint32_t(b)) << 21) | uint64_t(uint32_t(c));
  }
  uint32_t flat(int a, int b, int c) const { return (uint32_t(a) * nl + b) * nl + c; }

  void add_scaled(Acc& acc, uint32_t key, uint32_t pid, double s, int times_code) {
    Coef& dst = acc.at(key);
    const Coef& src = pool.at(pid);
    const int ns = pool.nslots.load(std::memory_order_acquire);
    for (int q = 0; q < ns; ++q) {
      if (src[q] == 0.0) continue;
      int code = pool.code_of_slot[q];
      if (times_code) {
        code = PolyPool::add_codes(code, times_code);
        if (code < 0) throw std::runtime_error("monomial degree overflow");
      }
      dst[pool.slot(code)] += s * src[q];
    }
  }

  // Adds s * (c_d if times_code) * T_kappa reduced into b_nl to acc.
  void add_reduced(Acc& acc, int a, int b, int c, double s, int times_code) {
    if (a < nl && b < nl && c < nl) {
      add_scaled(acc, flat(a, b, c), one_pid, s, times_code);
      return;
    }
    const SVec& r = red(a, b, c);
    for (const auto& [key, pid] : r) add_scaled(acc, key, pid, s, times_code);
  }

  // Reduction of T_kappa (kappa dominant, some coordinate >= nl) modulo
  // <T_{nl e_d} - c_d> into b_nl.
  const SVec& red(int a, int b, int c) {
    uint64_t key = key3(a, b, c);
    auto it = red_memo.find(key);
    if (it != red_memo.end()) return it->second;
    int k[3] = {a, b, c};
    int d = k[0] >= nl ? 0 : (k[1] >= nl ? 1 : 2);
    int mu[3] = {a, b, c};
    mu[d] -= nl;
    std::vector<std::array<int, 3>> terms;
    int cnt = 0;
    for (const auto& nu : orbit_e[d]) {
      int t0 = mu[0] + nl * nu[0], t1 = mu[1] + nl * nu[1], t2 = mu[2] + nl * nu[2];
      dominant(t0, t1, t2);
      if (t0 == a && t1 == b && t2 == c)
        ++cnt;
      else
        terms.push_back({t0, t1, t2});
    }
    if (cnt == 0) throw std::logic_error("reduction: leading term missing");
    Acc acc;
    const int cd_code = (d == 0) ? 1 : (d == 1 ? 4 : 16);
    add_reduced(acc, mu[0], mu[1], mu[2], double(orbit_e[d].size()) / cnt, cd_code);
    for (const auto& t : terms) add_reduced(acc, t[0], t[1], t[2], -1.0 / cnt, 0);
    SVec out = acc.finish(pool);
    return red_memo.emplace(key, std::move(out)).first->second;
  }

  // Column (def, abc) of C: coefficients of T_abc * T_{m def} in b_nl.
  SVec c_column(int f, int a, int b, int c, Acc& acc) {
    acc.clear();
    for (const auto& nu : orbit_def[f]) {
      int t0 = a + m * nu[0], t1 = b + m * nu[1], t2 = c + m * nu[2];
      dominant(t0, t1, t2);
      add_reduced(acc, t0, t1, t2, 1.0 / 24.0, 0);
    }
    return acc.finish(pool);
  }

  static int height(int a, int b, int c) { return 3 * a + 4 * b + 3 * c; }
};

// Runs body(i) for i in [0, count) on all hardware threads.
template <typename F>
void parallel_for(size_t count, F body) {
  unsigned nt = std::max(1u, std::min(std::thread::hardware_concurrency(), 64u));
  if (count < 2 * size_t(nt) || nt == 1) {
    for (size_t i = 0; i < count; ++i) body(i, 0u);
    return;
  }
  std::atomic<size_t> next{0};
  std::vector<std::thread> th;
  std::exception_ptr err;
  std::mutex err_mu;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      try {
        const size_t chunk = 256;
        for (;;) {
          size_t i0 = next.fetch_add(chunk);
          if (i0 >= count) break;
          for (size_t i = i0; i < std::min(count, i0 + chunk); ++i) body(i, t);
        }
      } catch (...) {
        std::lock_guard<std::mutex> lock(err_mu);
        err = std::current_exception();
      }
    });
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

std::unique_ptr<LevelTables> derive(int nl) {
  auto T = std::make_unique<LevelTables>();
  PolyPool pool;
  const int m = nl / 2;
  const uint32_t N = uint32_t(nl) * nl * nl;
  T->nl = nl;
  T->m = m;
  const unsigned nt = std::max(1u, std::min(std::thread::hardware_concurrency(), 64u));
  std::vector<std::unique_ptr<Deriver>> der;
  for (unsigned t = 0; t < nt; ++t) der.emplace_back(new Deriver(nl, pool));
  auto flat = [&](int a, int b, int c) { return (uint32_t(a) * nl + b) * nl + c; };

  // Phase 1: the C column of every kappa (kappa = abc + m def), in parallel.
  std::vector<SVec> ccol(N), bcol(N);
  parallel_for(N, [&](size_t k, unsigned t) {
    thread_local Acc acc;
    int ka = int(k / (uint32_t(nl) * nl)), kb = int((k / nl) % nl), kc = int(k % nl);
    int f = ((ka / m) << 2) | ((kb / m) << 1) | (kc / m);
    ccol[k] = der[t]->c_column(f, ka % m, kb % m, kc % m, acc);
  });
  der.clear();

  // Phase 2: B columns in increasing height; kappas of equal height are
  // independent, so each height class runs in parallel.
  const int hmax = 10 * (nl - 1);
  std::vector<uint32_t> order(N), start(hmax + 2, 0);
  for (int a = 0; a < nl; ++a)
    for (int b = 0; b < nl; ++b)
      for (int c = 0; c < nl; ++c) ++start[Deriver::height(a, b, c) + 1];
  for (int h = 0; h <= hmax; ++h) start[h + 1] += start[h];
  {
    std::vector<uint32_t> fill(start.begin(), start.end() - 1);
    for (int a = 0; a < nl; ++a)
      for (int b = 0; b < nl; ++b)
        for (int c = 0; c < nl; ++c) order[fill[Deriver::height(a, b, c)]++] = flat(a, b, c);
  }
  std::vector<uint8_t> done(N, 0);
  auto b_column = [&](uint32_t k, Acc& acc) {
      int ka = k / (nl * nl), kb = (k / nl) % nl, kc = k % nl;
      int f = ((ka / m) << 2) | ((kb / m) << 1) | (kc / m);
      int a = ka % m, b = kb % m, c = kc % m;
      const SVec& col = ccol[k];
      double d0 = 0.0;
      for (const auto& [key, pid] : col)
        if (key == k) {
          const Coef& p = pool.at(pid);
          for (int q = 1; q < K; ++q)
            if (p[q] != 0.0) throw std::logic_error("non-constant leading coefficient");
          d0 = p[0];
        }
      if (d0 == 0.0) throw std::logic_error("missing leading term");
      // position of b~_(def,abc) in the node-local interleaved layout
      uint32_t pos = flat(((f >> 2) & 1) + 2 * a, ((f >> 1) & 1) + 2 * b, (f & 1) + 2 * c);
      acc.clear();
      Coef lead{};
      lead[0] = 1.0 / d0;
      acc.at(pos) = lead;
      const int ns = pool.nslots.load(std::memory_order_acquire);
      for (const auto& [key, pid] : col) {
        if (key == k) continue;
        if (!done[key]) throw std::logic_error("height order violated");
        const Coef& P = pool.at(pid);
        for (const auto& [row, qid] : bcol[key]) {
          const Coef& Q = pool.at(qid);
          Coef& dst = acc.at(row);
          for (int s1 = 0; s1 < ns; ++s1) {
            if (P[s1] == 0.0) continue;
            for (int s2 = 0; s2 < ns; ++s2) {
              if (Q[s2] == 0.0) continue;
              int code = PolyPool::add_codes(pool.code_of_slot[s1], pool.code_of_slot[s2]);
              if (code < 0) throw std::runtime_error("monomial degree overflow");
              dst[pool.slot(code)] -= P[s1] * Q[s2] / d0;
            }
          }
        }
      }
      bcol[k] = acc.finish(pool);
    done[k] = 1;
  };
  // persistent workers; a spin barrier separates height classes
  std::atomic<int> arrived{0};
  std::atomic<int> phase{0};
  std::atomic<size_t> next{0};
  std::atomic<bool> failed{false};
  std::exception_ptr err;
  std::mutex err_mu;
  auto worker = [&](unsigned t) {
    Acc acc;
    int my_phase = 0;
    for (int h = 0; h <= hmax; ++h) {
      const size_t n0 = start[h], n1 = start[h + 1];
      try {
        for (;;) {
          if (failed.load(std::memory_order_relaxed)) break;
          size_t i = next.fetch_add(1);
          if (i >= n1 - n0) break;
          b_column(order[n0 + i], acc);
        }
      } catch (...) {
        std::lock_guard<std::mutex> lock(err_mu);
        err = std::current_exception();
        failed.store(true);
      }
      // barrier: the last thread to arrive resets the work counter
      if (arrived.fetch_add(1) == int(nt) - 1) {
        arrived.store(0);
        next.store(0);
        phase.fetch_add(1, std::memory_order_release);
      } else {
        while (phase.load(std::memory_order_acquire) == my_phase) std::this_thread::yield();
      }
      ++my_phase;
    }
    (void)t;
  };
  {
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(worker, t);
    worker(0);
    for (auto& x : th) x.join();
  }
  if (err) std::rethrow_exception(err);

  // ---- gather tables (parallel transpose; rows sorted for a deterministic order)
  auto cube_row = [&](uint32_t pos) {  // node-local position -> table row
    int x = int(pos / (uint32_t(nl) * nl)), y = int((pos / nl) % nl), z = int(pos % nl);
    int cube = ((x >> 1) * m + (y >> 1)) * m + (z >> 1);
    return cube * 8 + (((x & 1) << 2) | ((y & 1) << 1) | (z & 1));
  };
  auto c_src_of = [&](uint32_t k) {  // position def + 2 abc of the C column of kappa
    int ka = k / (nl * nl), kb = (k / nl) % nl, kc = k % nl;
    int f = ((ka / m) << 2) | ((kb / m) << 1) | (kc / m);
    return pack3(((f >> 2) & 1) + 2 * (ka % m), ((f >> 1) & 1) + 2 * (kb % m), (f & 1) + 2 * (kc % m));
  };
  const int rows = 8 * m * m * m;  // == N
  T->b_rowptr.assign(rows + 1, 0);
  T->c_rowptr.assign(rows + 1, 0);
  std::vector<uint8_t> used(pool.count.load(), 0);
  parallel_for(N, [&](size_t k, unsigned) {
    for (const auto& [pos, pid] : bcol[k]) {
      __atomic_fetch_add(&T->b_rowptr[cube_row(pos) + 1], 1, __ATOMIC_RELAXED);
      used[pid] = 1;
    }
    for (const auto& [kk, pid] : ccol[k]) {
      __atomic_fetch_add(&T->c_rowptr[cube_row(kk) + 1], 1, __ATOMIC_RELAXED);
      used[pid] = 1;
    }
  });
  for (int r = 0; r < rows; ++r) {
    T->b_rowptr[r + 1] += T->b_rowptr[r];
    T->c_rowptr[r + 1] += T->c_rowptr[r];
  }
  // Canonical numbering (pool ids and slot order depend on thread timing):
  // monomials by code, polynomials by their coefficient vectors in that order.
  std::vector<uint32_t> live;
  for (uint32_t p = 0; p < used.size(); ++p)
    if (used[p]) live.push_back(p);
  std::vector<int> slots;
  {
    std::vector<int> slot_used(K, 0);
    slot_used[0] = 1;
    for (uint32_t p : live)
      for (int q = 0; q < K; ++q)
        if (pool.at(p)[q] != 0.0) slot_used[q] = 1;
    for (int q = 0; q < (int)pool.nslots.load(); ++q)
      if (slot_used[q]) slots.push_back(q);
    std::sort(slots.begin(), slots.end(), [&](int a, int b) { return pool.code_of_slot[a] < pool.code_of_slot[b]; });
  }
  auto canon = [&](uint32_t p) {
    std::vector<long long> v;
    for (int q : slots) v.push_back(std::llround(pool.at(p)[q] * 1073741824.0));
    return v;
  };
  std::sort(live.begin(), live.end(), [&](uint32_t a, uint32_t b) { return canon(a) < canon(b); });
  std::vector<uint32_t> remap(used.size(), 0xffffffffu);
  for (uint32_t i = 0; i < live.size(); ++i) remap[live[i]] = i;
  const uint32_t npoly = uint32_t(live.size());
  T->b_src.resize(T->b_rowptr[rows]);
  T->b_pid.resize(T->b_rowptr[rows]);
  T->c_src.resize(T->c_rowptr[rows]);
  T->c_pid.resize(T->c_rowptr[rows]);
  {
    std::vector<int> bfill(T->b_rowptr.begin(), T->b_rowptr.end() - 1);
    std::vector<int> cfill(T->c_rowptr.begin(), T->c_rowptr.end() - 1);
    parallel_for(N, [&](size_t k, unsigned) {
      const uint32_t bsrc = pack3(int(k / (uint32_t(nl) * nl)), int((k / nl) % nl), int(k % nl));
      for (const auto& [pos, pid] : bcol[k]) {
        int q = __atomic_fetch_add(&bfill[cube_row(pos)], 1, __ATOMIC_RELAXED);
        T->b_src[q] = bsrc;
        T->b_pid[q] = (uint16_t)remap[pid];
      }
      const uint32_t csrc = c_src_of(uint32_t(k));
      for (const auto& [kk, pid] : ccol[k]) {
        int q = __atomic_fetch_add(&cfill[cube_row(kk)], 1, __ATOMIC_RELAXED);
        T->c_src[q] = csrc;
        T->c_pid[q] = (uint16_t)remap[pid];
      }
    });
  }
  auto sort_rows = [&](const std::vector<int>& rp, std::vector<uint32_t>& src, std::vector<uint16_t>& pid) {
    parallel_for(size_t(rows), [&](size_t r, unsigned) {
      const int a = rp[r], b = rp[r + 1];
      std::pair<uint32_t, uint16_t> tmp[64];
      std::vector<std::pair<uint32_t, uint16_t>> big;
      std::pair<uint32_t, uint16_t>* e = tmp;
      if (b - a > 64) {
        big.resize(b - a);
        e = big.data();
      }
      for (int i = a; i < b; ++i) e[i - a] = {src[i], pid[i]};
      std::sort(e, e + (b - a));
      for (int i = a; i < b; ++i) {
        src[i] = e[i - a].first;
        pid[i] = e[i - a].second;
      }
    });
  };
  sort_rows(T->b_rowptr, T->b_src, T->b_pid);
  sort_rows(T->c_rowptr, T->c_src, T->c_pid);
  std::vector<SVec>().swap(bcol);
  std::vector<SVec>().swap(ccol);
  if (npoly > 65535) throw std::runtime_error("too many coefficient polynomials");
  T->nmono = (int)slots.size();
  for (int q : slots) {
    int code = pool.code_of_slot[q];
    T->mono.push_back(code % 4);
    T->mono.push_back((code / 4) % 4);
    T->mono.push_back(code / 16);
  }
  T->npoly = (int)npoly;
  T->poly.assign(size_t(npoly) * T->nmono, 0.0);
  for (uint32_t i = 0; i < npoly; ++i)
    for (int q = 0; q < T->nmono; ++q) T->poly[size_t(i) * T->nmono + q] = pool.at(live[i])[slots[q]];
  return T;
}

}  // namespace

const LevelTables* level_tables(int nl) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<LevelTables>> cache;
  if (nl < 2 || nl > 1024 || (nl & (nl - 1))) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(nl);
  if (it != cache.end()) return it->second.get();
  try {
    auto t = derive(nl);
    return cache.emplace(nl, std::move(t)).first->second.get();
  } catch (const std::bad_alloc&) {
    return nullptr;
  }
}

const GatherBlocks* gather_blocks(int nl) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<GatherBlocks>> cache;
  const LevelTables* T = level_tables(nl);
  if (!T) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(nl);
  if (it != cache.end()) return it->second.get();
  try {
    const int m = T->m, cubes = m * m * m;
    const auto& rp = T->b_rowptr;
    const auto& src = T->b_src;
    auto flat = [&](uint32_t s) { return (size_t(s >> 20) * nl + ((s >> 10) & 1023u)) * nl + (s & 1023u); };
    // union-find over cubes; the root of a set is its smallest cube
    std::vector<int> par(cubes);
    for (int c = 0; c < cubes; ++c) par[c] = c;
    auto find = [&](int x) {
      while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
      }
      return x;
    };
    auto out = std::make_unique<GatherBlocks>();
    std::vector<int>& owner = out->kappa;  // first cube that reads a source, then its block
    owner.assign(size_t(nl) * nl * nl, -1);
    for (int c = 0; c < cubes; ++c)
      for (int e = rp[size_t(c) * 8]; e < rp[size_t(c) * 8 + 8]; ++e) {
        const size_t k = flat(src[e]);
        if (owner[k] < 0) {
          owner[k] = c;
        } else {
          const int a = find(owner[k]), b = find(c);
          if (a != b) par[std::max(a, b)] = std::min(a, b);
        }
      }
    out->cube.resize(cubes);
    for (int c = 0; c < cubes; ++c) out->cube[c] = find(c);
    for (int& o : owner)
      if (o >= 0) o = out->cube[o];
    return cache.emplace(nl, std::move(out)).first->second.get();
  } catch (const std::bad_alloc&) {
    return nullptr;
  }
}

}  // namespace fcc
