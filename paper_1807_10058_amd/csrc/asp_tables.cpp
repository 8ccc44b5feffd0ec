// Derivation of the B_nl / C_nl gather tables; see asp_tables.hpp for the
// mathematics and the paper passages it follows.
#include "asp_tables.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
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

struct PolyPool {
  int slot_of_code[64];
  std::vector<int> code_of_slot;
  std::vector<Coef> polys;
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
  std::unordered_map<QKey, uint32_t, QHash> index;
  PolyPool() {
    std::fill(std::begin(slot_of_code), std::end(slot_of_code), -1);
    slot(0);  // the constant monomial is slot 0
  }
  int slot(int code) {
    if (slot_of_code[code] < 0) {
      if ((int)code_of_slot.size() >= K) throw std::runtime_error("too many monomials");
      slot_of_code[code] = (int)code_of_slot.size();
      code_of_slot.push_back(code);
    }
    return slot_of_code[code];
  }
  uint32_t intern(const Coef& p) {
    QKey key;
    for (int i = 0; i < K; ++i) key.q[i] = std::llround(p[i] * 1073741824.0);  // 2^30
    auto it = index.find(key);
    if (it != index.end()) return it->second;
    uint32_t id = (uint32_t)polys.size();
    polys.push_back(p);
    index.emplace(std::move(key), id);
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
  Coef& at(uint32_t key) {
    for (size_t i = 0; i < keys.size(); ++i)
      if (keys[i] == key) return vals[i];
    keys.push_back(key);
    vals.push_back(Coef{});
    return vals.back();
  }
  SVec finish(PolyPool& pool) {
    SVec out;
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

struct Deriver {
  int nl, m;
  PolyPool pool;
  std::array<std::vector<std::array<int, 3>>, 3> orbit_e;   // distinct W e_d
  std::array<std::vector<std::array<int, 3>>, 8> orbit_def; // g def for all 24 g
  std::unordered_map<uint64_t, SVec> red_memo;

  explicit Deriver(int nl_) : nl(nl_), m(nl_ / 2) {
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
  }
  static uint64_t key3(int a, int b, int c) {
    return (uint64_t(uint32_t(a)) << 42) | (uint64_t(uint32_t(b)) << 21) | uint64_t(uint32_t(c));
  }
  uint32_t flat(int a, int b, int c) const { return (uint32_t(a) * nl + b) * nl + c; }

  void add_scaled(Acc& acc, const SVec& v, double s, int times_code) {
    for (const auto& [key, pid] : v) {
      Coef& dst = acc.at(key);
      const Coef src = pool.polys[pid];
      for (int q = 0; q < (int)pool.code_of_slot.size(); ++q) {
        if (src[q] == 0.0) continue;
        int code = pool.code_of_slot[q];
        if (times_code) {
          code = PolyPool::add_codes(code, times_code);
          if (code < 0) throw std::runtime_error("monomial degree overflow");
        }
        dst[pool.slot(code)] += s * src[q];
      }
    }
  }

  // Reduction of T_kappa (kappa dominant) modulo <T_{nl e_d} - c_d> into b_nl.
  const SVec& red(int a, int b, int c) {
    uint64_t key = key3(a, b, c);
    auto it = red_memo.find(key);
    if (it != red_memo.end()) return it->second;
    SVec out;
    if (a < nl && b < nl && c < nl) {
      Coef one{};
      one[0] = 1.0;
      out.emplace_back(flat(a, b, c), pool.intern(one));
    } else {
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
      {
        const SVec& r = red(mu[0], mu[1], mu[2]);  // node-based map: reference stays valid
        add_scaled(acc, r, double(orbit_e[d].size()) / cnt, cd_code);
      }
      for (const auto& t : terms) {
        add_scaled(acc, red(t[0], t[1], t[2]), -1.0 / cnt, 0);
      }
      out = acc.finish(pool);
    }
    return red_memo.emplace(key, std::move(out)).first->second;
  }

  // Column (def, abc) of C: coefficients of T_abc * T_{m def} in b_nl.
  SVec c_column(int f, int a, int b, int c) {
    Acc acc;
    for (const auto& nu : orbit_def[f]) {
      int t0 = a + m * nu[0], t1 = b + m * nu[1], t2 = c + m * nu[2];
      dominant(t0, t1, t2);
      add_scaled(acc, red(t0, t1, t2), 1.0 / 24.0, 0);
    }
    return acc.finish(pool);
  }

  static int height(int a, int b, int c) { return 3 * a + 4 * b + 3 * c; }
};

std::unique_ptr<LevelTables> derive(int nl) {
  auto T = std::make_unique<LevelTables>();
  Deriver D(nl);
  const int m = nl / 2;
  const uint32_t N = uint32_t(nl) * nl * nl;
  T->nl = nl;
  T->m = m;
  // Per kappa: its C column (kappa = abc + m def) and its B column.
  std::vector<SVec> ccol(N), bcol(N);
  std::vector<uint8_t> done(N, 0);
  // kappa in increasing height (counting sort)
  const int hmax = 10 * (nl - 1);
  std::vector<uint32_t> order(N), count(hmax + 2, 0);
  for (int a = 0; a < nl; ++a)
    for (int b = 0; b < nl; ++b)
      for (int c = 0; c < nl; ++c) ++count[Deriver::height(a, b, c) + 1];
  for (int h = 0; h <= hmax; ++h) count[h + 1] += count[h];
  for (int a = 0; a < nl; ++a)
    for (int b = 0; b < nl; ++b)
      for (int c = 0; c < nl; ++c) order[count[Deriver::height(a, b, c)]++] = D.flat(a, b, c);

  for (uint32_t k : order) {
    int ka = k / (nl * nl), kb = (k / nl) % nl, kc = k % nl;
    int f = ((ka / m) << 2) | ((kb / m) << 1) | (kc / m);
    int a = ka % m, b = kb % m, c = kc % m;
    SVec col = D.c_column(f, a, b, c);
    // leading coefficient (constant) on kappa itself
    double d0 = 0.0;
    for (const auto& [key, pid] : col)
      if (key == k) {
        const Coef& p = D.pool.polys[pid];
        for (int q = 1; q < K; ++q)
          if (p[q] != 0.0) throw std::logic_error("non-constant leading coefficient");
        d0 = p[0];
      }
    if (d0 == 0.0) throw std::logic_error("missing leading term");
    // position of b~_(def,abc) in the node-local interleaved layout
    uint32_t pos = D.flat(((f >> 2) & 1) + 2 * a, ((f >> 1) & 1) + 2 * b, (f & 1) + 2 * c);
    Acc acc;
    Coef lead{};
    lead[0] = 1.0 / d0;
    acc.at(pos) = lead;
    for (const auto& [key, pid] : col) {
      if (key == k) continue;
      if (!done[key]) throw std::logic_error("height order violated");
      const Coef P = D.pool.polys[pid];
      for (const auto& [row, qid] : bcol[key]) {
        const Coef Q = D.pool.polys[qid];
        Coef& dst = acc.at(row);
        for (int s = 0; s < (int)D.pool.code_of_slot.size(); ++s) {
          if (P[s] == 0.0) continue;
          for (int t = 0; t < (int)D.pool.code_of_slot.size(); ++t) {
            if (Q[t] == 0.0) continue;
            int code = PolyPool::add_codes(D.pool.code_of_slot[s], D.pool.code_of_slot[t]);
            if (code < 0) throw std::runtime_error("monomial degree overflow");
            dst[D.pool.slot(code)] -= P[s] * Q[t] / d0;
          }
        }
      }
    }
    bcol[k] = acc.finish(D.pool);
    ccol[k] = std::move(col);
    done[k] = 1;
  }
  D.red_memo.clear();

  // ---- gather tables ----------------------------------------------------
  auto cube_row = [&](int x, int y, int z) {  // node-local position -> table row
    int cube = ((x >> 1) * m + (y >> 1)) * m + (z >> 1);
    return cube * 8 + (((x & 1) << 2) | ((y & 1) << 1) | (z & 1));
  };
  const int rows = 8 * m * m * m;  // == N
  T->b_rowptr.assign(rows + 1, 0);
  T->c_rowptr.assign(rows + 1, 0);
  // B: column kappa, entry (pos, pid) -> row cube_row(pos), source kappa
  for (uint32_t k = 0; k < N; ++k)
    for (const auto& [pos, pid] : bcol[k]) ++T->b_rowptr[cube_row(pos / (nl * nl), (pos / nl) % nl, pos % nl) + 1];
  // C: column at pos(kappa), entry (kappa', pid) -> row cube_row(kappa'), source pos
  for (uint32_t k = 0; k < N; ++k)
    for (const auto& [kk, pid] : ccol[k]) ++T->c_rowptr[cube_row(kk / (nl * nl), (kk / nl) % nl, kk % nl) + 1];
  for (int r = 0; r < rows; ++r) {
    T->b_rowptr[r + 1] += T->b_rowptr[r];
    T->c_rowptr[r + 1] += T->c_rowptr[r];
  }
  T->b_src.resize(T->b_rowptr[rows]);
  T->b_pid.resize(T->b_rowptr[rows]);
  T->c_src.resize(T->c_rowptr[rows]);
  T->c_pid.resize(T->c_rowptr[rows]);
  std::vector<uint32_t> used(D.pool.polys.size(), 0xffffffffu);
  uint32_t npoly = 0;
  auto remap = [&](uint32_t pid) {
    if (used[pid] == 0xffffffffu) used[pid] = npoly++;
    return used[pid];
  };
  {
    std::vector<int> fill(T->b_rowptr.begin(), T->b_rowptr.end() - 1);
    for (uint32_t k = 0; k < N; ++k) {
      uint32_t src = pack3(k / (nl * nl), (k / nl) % nl, k % nl);
      for (const auto& [pos, pid] : bcol[k]) {
        int r = cube_row(pos / (nl * nl), (pos / nl) % nl, pos % nl);
        T->b_src[fill[r]] = src;
        T->b_pid[fill[r]++] = (uint16_t)remap(pid);
      }
    }
  }
  {
    std::vector<int> fill(T->c_rowptr.begin(), T->c_rowptr.end() - 1);
    for (uint32_t k = 0; k < N; ++k) {
      int ka = k / (nl * nl), kb = (k / nl) % nl, kc = k % nl;
      int f = ((ka / m) << 2) | ((kb / m) << 1) | (kc / m);
      uint32_t src = pack3(((f >> 2) & 1) + 2 * (ka % m), ((f >> 1) & 1) + 2 * (kb % m), (f & 1) + 2 * (kc % m));
      for (const auto& [kk, pid] : ccol[k]) {
        int r = cube_row(kk / (nl * nl), (kk / nl) % nl, kk % nl);
        T->c_src[fill[r]] = src;
        T->c_pid[fill[r]++] = (uint16_t)remap(pid);
      }
    }
  }
  if (npoly > 65535) throw std::runtime_error("too many coefficient polynomials");
  // monomials actually used
  std::vector<int> slot_used(K, 0);
  for (uint32_t p = 0; p < D.pool.polys.size(); ++p)
    if (used[p] != 0xffffffffu)
      for (int s = 0; s < K; ++s)
        if (D.pool.polys[p][s] != 0.0) slot_used[s] = 1;
  slot_used[0] = 1;
  std::vector<int> slots;
  for (int s = 0; s < (int)D.pool.code_of_slot.size(); ++s)
    if (slot_used[s]) slots.push_back(s);
  T->nmono = (int)slots.size();
  for (int s : slots) {
    int code = D.pool.code_of_slot[s];
    T->mono.push_back(code % 4);
    T->mono.push_back((code / 4) % 4);
    T->mono.push_back(code / 16);
  }
  T->npoly = (int)npoly;
  T->poly.assign(size_t(npoly) * T->nmono, 0.0);
  for (uint32_t p = 0; p < D.pool.polys.size(); ++p)
    if (used[p] != 0xffffffffu)
      for (int q = 0; q < T->nmono; ++q) T->poly[size_t(used[p]) * T->nmono + q] = D.pool.polys[p][slots[q]];
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

}  // namespace fcc
