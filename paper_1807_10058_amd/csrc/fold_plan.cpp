// Unfold tables of the fold+FFT formulation (see fold_plan.hpp for the
// derivation).  Every point k gets the signature of its orbit: for each u in
// W the wrap floor(u k / n) and the first u' with u' k = u k mod n.  Points of
// equal signature have equal unfold rows, so the Gram block solve runs once
// per signature and the rows are shared.
#include "fold_plan.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <thread>
#include <unordered_map>

namespace fcc {
namespace {

using cd = std::complex<double>;

struct Group {
  int g[24][9];
  int inv[24];
};
const Group& group() {
  static const Group G = [] {
    Group r{};
#define FCC_G(u, a0, a1, a2, a3, a4, a5, a6, a7, a8, ui) \
  {                                                     \
    const int m[9] = {a0, a1, a2, a3, a4, a5, a6, a7, a8}; \
    std::copy(m, m + 9, r.g[u]);                        \
    r.inv[u] = ui;                                      \
  }
#include "orbits.inc"
    FCC_GROUP(FCC_G)
#undef FCC_G
    return r;
  }();
  return G;
}

inline void act(const int* g, const long long v[3], long long o[3]) {
  for (int i = 0; i < 3; ++i) o[i] = g[3 * i] * v[0] + g[3 * i + 1] * v[1] + g[3 * i + 2] * v[2];
}

cd omega8(long long m) {  // exp(2 pi i m / 8)
  static const double h = std::sqrt(0.5);
  static const cd t[8] = {{1, 0}, {h, h}, {0, 1}, {-h, h}, {-1, 0}, {-h, -h}, {0, -1}, {h, -h}};
  return t[((m % 8) + 8) % 8];
}

using Key = std::array<uint64_t, 6>;
struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = 1469598103934665603ull;
    for (uint64_t w : k) {
      h ^= w;
      h *= 1099511628211ull;
      h ^= h >> 29;
    }
    return size_t(h);
  }
};

struct Builder {
  int n, lg;
  int r8[3];
  cd Ttab[7][7][7];  // T_r(rst) for r in [-3, 3]^3
  std::map<std::vector<long long>, int> rows;
  std::vector<cd> K;
  fcc_status err = FCC_OK;

  // wraps and reduced points of u k for every u
  void orbit(const long long k[3], long long fl[24][3], long long flat[24]) const {
    const Group& G = group();
    for (int u = 0; u < 24; ++u) {
      long long v[3];
      act(G.g[u], k, v);
      long long m[3];
      for (int i = 0; i < 3; ++i) {
        fl[u][i] = ((v[i] + 4LL * n) >> lg) - 4;  // |v| < 3n
        m[i] = v[i] - fl[u][i] * n;
      }
      flat[u] = (m[0] * n + m[1]) * n + m[2];
    }
  }
  Key signature(const long long k[3]) const {
    long long fl[24][3], flat[24];
    orbit(k, fl, flat);
    Key key{};
    for (int u = 0; u < 24; ++u) {
      int first = u;
      for (int v = 0; v < u; ++v)
        if (flat[v] == flat[u]) {
          first = v;
          break;
        }
      const uint64_t code = uint64_t(fl[u][0] + 3) | (uint64_t(fl[u][1] + 3) << 3) | (uint64_t(fl[u][2] + 3) << 6) |
                            (uint64_t(first) << 9);
      key[u / 4] |= code << (14 * (u % 4));
    }
    return key;
  }
  cd T(const long long r[3]) const {
    for (int i = 0; i < 3; ++i)
      if (r[i] < -3 || r[i] > 3) {
        // not reached for |u k| < 3n; evaluate directly
        cd s = 0;
        const Group& G = group();
        for (int g = 0; g < 24; ++g) {
          long long v[3];
          act(G.g[g], r, v);
          s += omega8(v[0] * r8[0] + v[1] * r8[1] + v[2] * r8[2]);
        }
        return s / 24.0;
      }
    return Ttab[r[0] + 3][r[1] + 3][r[2] + 3];
  }
  // Gram row of point k: (flat target, value) with the wraps rho_u = -floor(u k / n)
  void gram_row(const long long k[3], std::vector<std::pair<long long, cd>>& row) const {
    long long fl[24][3], flat[24];
    orbit(k, fl, flat);
    row.clear();
    for (int u = 0; u < 24; ++u) {
      const long long rho[3] = {-fl[u][0], -fl[u][1], -fl[u][2]};
      const cd v = T(rho) / 24.0;
      auto it = std::find_if(row.begin(), row.end(), [&](const auto& e) { return e.first == flat[u]; });
      if (it == row.end())
        row.push_back({flat[u], v});
      else
        it->second += v;
    }
  }
  // The unfold row K_k of eq. (2) for point k; -1 on failure (err set).
  int solve(const long long k[3]) {
    const Group& G = group();
    auto coords = [&](long long f, long long c[3]) {
      c[0] = f / ((long long)n * n);
      c[1] = (f / n) % n;
      c[2] = f % n;
    };
    std::vector<long long> mem{(k[0] * n + k[1]) * n + k[2]};
    std::vector<std::vector<std::pair<long long, cd>>> grow;
    for (size_t i = 0; i < mem.size(); ++i) {
      long long c[3];
      coords(mem[i], c);
      std::vector<std::pair<long long, cd>> row;
      gram_row(c, row);
      for (const auto& e : row)
        if (std::abs(e.second) > 1e-12 && std::find(mem.begin(), mem.end(), e.first) == mem.end()) mem.push_back(e.first);
      grow.push_back(std::move(row));
      if (mem.size() > 24) {
        err = FCC_ERR_UNSUPPORTED;
        return -1;
      }
    }
    const int s = int(mem.size());
    // [M | I] -> [I | M^{-1}], partial pivoting; M = 24 Gram restricted to the block
    std::vector<cd> a(size_t(s) * 2 * s, 0.0);
    for (int i = 0; i < s; ++i) {
      for (const auto& e : grow[i]) {
        const int j = int(std::find(mem.begin(), mem.end(), e.first) - mem.begin());
        if (j < s) a[size_t(i) * 2 * s + j] = 24.0 * e.second;
      }
      a[size_t(i) * 2 * s + s + i] = 1.0;
    }
    for (int c = 0; c < s; ++c) {
      int p = c;
      for (int r = c + 1; r < s; ++r)
        if (std::abs(a[size_t(r) * 2 * s + c]) > std::abs(a[size_t(p) * 2 * s + c])) p = r;
      if (std::abs(a[size_t(p) * 2 * s + c]) < 1e-9) {
        err = FCC_ERR_SINGULAR_SKEW;
        return -1;
      }
      for (int j = 0; j < 2 * s; ++j) std::swap(a[size_t(c) * 2 * s + j], a[size_t(p) * 2 * s + j]);
      const cd d = a[size_t(c) * 2 * s + c];
      for (int j = 0; j < 2 * s; ++j) a[size_t(c) * 2 * s + j] /= d;
      for (int r = 0; r < s; ++r) {
        if (r == c) continue;
        const cd f = a[size_t(r) * 2 * s + c];
        if (f == cd(0)) continue;
        for (int j = 0; j < 2 * s; ++j) a[size_t(r) * 2 * s + j] -= f * a[size_t(c) * 2 * s + j];
      }
    }
    // Gram^{-1}[k, m_j] = 24 (M^{-1})[0, j]
    long long fl[24][3], flat[24];
    orbit(k, fl, flat);
    cd Kr[24] = {};
    for (int j = 0; j < s; ++j) {
      const cd c = 24.0 * a[size_t(0) * 2 * s + s + j];
      if (std::abs(c) < 1e-13) continue;
      int h = 0;
      while (h < 24 && flat[h] != mem[j]) ++h;
      if (h == 24) {  // a Gram block reaches outside the orbit: not a fold block
        err = FCC_ERR_UNSUPPORTED;
        return -1;
      }
      const long long rho[3] = {-fl[h][0], -fl[h][1], -fl[h][2]};
      long long v[3];
      act(G.g[G.inv[h]], rho, v);
      for (int u = 0; u < 24; ++u) {
        long long w[3];
        act(G.g[u], v, w);
        Kr[u] += c * std::conj(omega8(w[0] * r8[0] + w[1] * r8[1] + w[2] * r8[2])) / 24.0;
      }
    }
    std::vector<long long> key(48);
    for (int u = 0; u < 24; ++u) {
      key[2 * u] = std::llround(Kr[u].real() * 68719476736.0);
      key[2 * u + 1] = std::llround(Kr[u].imag() * 68719476736.0);
    }
    auto it = rows.find(key);
    if (it != rows.end()) return it->second;
    const int id = int(rows.size());
    if (id >= 256) {
      err = FCC_ERR_UNSUPPORTED;
      return -1;
    }
    rows.emplace(std::move(key), id);
    K.insert(K.end(), Kr, Kr + 24);
    return id;
  }
};

}  // namespace

fcc_status fold_tables(int n, const int r8[3], FoldTables* out, bool orbits) {
  if (n < 1 || (n & (n - 1)) || n > 1024 || !out) return FCC_ERR_INVALID_ARG;
  Builder b;
  b.n = n;
  b.lg = 0;
  while ((1 << b.lg) < n) ++b.lg;
  for (int i = 0; i < 3; ++i) b.r8[i] = r8[i];
  const Group& G = group();
  for (int x = -3; x <= 3; ++x)
    for (int y = -3; y <= 3; ++y)
      for (int z = -3; z <= 3; ++z) {
        cd s = 0;
        const long long r[3] = {x, y, z};
        for (int g = 0; g < 24; ++g) {
          long long v[3];
          act(G.g[g], r, v);
          s += omega8(v[0] * r8[0] + v[1] * r8[1] + v[2] * r8[2]);
        }
        b.Ttab[x + 3][y + 3][z + 3] = s / 24.0;
      }
  const long long N = (long long)n * n * n;
  std::vector<uint8_t> isrep;
  try {
    out->pid.assign(size_t(N), 0);
    if (orbits) isrep.assign(size_t(N), 0);
  } catch (const std::bad_alloc&) {
    return FCC_ERR_OOM;
  }
  // Deterministic in three passes: (1) in parallel, each point's wrap
  // signature, numbered per thread (pid holds the thread-local number for now)
  // with the thread's first point of every signature; (2) serially, every
  // signature solved once from its first point overall, signatures taken in
  // order of that point, so row numbers and values do not depend on thread
  // timing; (3) pid renumbered.
  const int nt = int(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  const int workers = N < 32768 ? 1 : nt;
  std::vector<std::vector<std::pair<Key, long long>>> firsts(workers);  // per thread: (signature, first point)
  std::vector<fcc_status> werr(workers, FCC_OK);
  auto work = [&](int t, long long lo, long long hi) {
    std::unordered_map<Key, int, KeyHash> local;
    for (long long f = lo; f < hi; ++f) {
      const long long k[3] = {f >> (2 * b.lg), (f >> b.lg) & (n - 1), f & (n - 1)};
      const Key key = b.signature(k);
      auto it = local.find(key);
      int id;
      if (it != local.end()) {
        id = it->second;
      } else {
        id = int(local.size());
        if (id > 255) {
          werr[t] = FCC_ERR_UNSUPPORTED;
          return;
        }
        local.emplace(key, id);
        firsts[t].push_back({key, f});
      }
      out->pid[size_t(f)] = uint8_t(id);
      if (orbits) {
        long long fl[24][3], flat[24];
        b.orbit(k, fl, flat);
        bool rep = true;
        for (int u = 1; u < 24 && rep; ++u) rep = flat[u] >= f;
        isrep[size_t(f)] = rep;
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < workers; ++t) th.emplace_back(work, t, N * t / workers, N * (t + 1) / workers);
  for (auto& t : th) t.join();
  for (fcc_status e : werr)
    if (e != FCC_OK) return e;
  // ranges are in increasing order, so a signature's first point overall is
  // its first point in the lowest thread that meets it
  std::unordered_map<Key, long long, KeyHash> first_all;
  for (int t = 0; t < workers; ++t)
    for (const auto& kf : firsts[t]) first_all.emplace(kf.first, kf.second);
  std::vector<std::pair<long long, Key>> order;
  for (const auto& kv : first_all) order.push_back({kv.second, kv.first});
  std::sort(order.begin(), order.end(), [](const auto& a, const auto& c) { return a.first < c.first; });
  std::unordered_map<Key, int, KeyHash> row_of;
  for (const auto& fk : order) {
    const long long f = fk.first;
    const long long k[3] = {f >> (2 * b.lg), (f >> b.lg) & (n - 1), f & (n - 1)};
    const int id = b.solve(k);
    if (id < 0) return b.err;
    row_of.emplace(fk.second, id);
  }
  std::vector<std::vector<uint8_t>> remap(workers);
  for (int t = 0; t < workers; ++t)
    for (const auto& kf : firsts[t]) remap[t].push_back(uint8_t(row_of.at(kf.first)));
  auto renumber = [&](int t, long long lo, long long hi) {
    for (long long f = lo; f < hi; ++f) out->pid[size_t(f)] = remap[t][out->pid[size_t(f)]];
  };
  th.clear();
  for (int t = 0; t < workers; ++t) th.emplace_back(renumber, t, N * t / workers, N * (t + 1) / workers);
  for (auto& t : th) t.join();
  if (b.err != FCC_OK) return b.err;
  out->K = std::move(b.K);
  out->npat = int(b.rows.size());
  if (orbits) {
    const int sa = std::min(n, kFoldBox[0]), sb = std::min(n, kFoldBox[1]), sc = std::min(n, kFoldBox[2]);
    const long long na = n / sa, nb = n / sb, nc = n / sc;
    out->reps.clear();
    for (long long B = 0; B < na * nb * nc; ++B) {
      const long long ba = B / (nb * nc), bb = (B / nc) % nb, bc = B % nc;
      for (int i = 0; i < sa; ++i)
        for (int j = 0; j < sb; ++j)
          for (int l = 0; l < sc; ++l) {
            const long long f = ((ba * sa + i) * n + (bb * sb + j)) * n + (bc * sc + l);
            if (isrep[size_t(f)]) out->reps.push_back(int32_t(f));
          }
    }
    const size_t nr = out->reps.size();
    try {
      out->prid.assign(24 * nr, 0);
    } catch (const std::bad_alloc&) {
      return FCC_ERR_OOM;
    }
    for (size_t r = 0; r < nr; ++r) {
      const long long f = out->reps[r];
      const long long k[3] = {f >> (2 * b.lg), (f >> b.lg) & (n - 1), f & (n - 1)};
      long long fl[24][3], flat[24];
      b.orbit(k, fl, flat);
      for (int h = 0; h < 24; ++h) out->prid[size_t(h) * nr + r] = out->pid[size_t(flat[h])];
    }
  }
  return FCC_OK;
}

}  // namespace fcc

extern "C" fcc_status fcc_fold_unfold_tables(int n, const double rst[3], unsigned char* pid, double* K, int* npat) {
  if (!pid || !K || !npat || !rst) return FCC_ERR_INVALID_ARG;
  int r8[3];
  for (int i = 0; i < 3; ++i) {
    const double v = 8.0 * rst[i];
    if (!std::isfinite(v) || std::fabs(v - std::nearbyint(v)) > 1e-12) return FCC_ERR_UNSUPPORTED;
    r8[i] = int(std::nearbyint(v));
  }
  fcc::FoldTables t;
  const fcc_status s = fcc::fold_tables(n, r8, &t);
  if (s != FCC_OK) return s;
  std::copy(t.pid.begin(), t.pid.end(), pid);
  for (size_t i = 0; i < t.K.size(); ++i) {
    K[2 * i] = t.K[i].real();
    K[2 * i + 1] = t.K[i].imag();
  }
  *npat = t.npat;
  return FCC_OK;
}
