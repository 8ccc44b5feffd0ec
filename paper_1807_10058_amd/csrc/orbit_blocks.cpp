// Orbit-block templates of the basis change; see orbit_blocks.hpp.
#include "orbit_blocks.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <thread>

#include "asp_tables.hpp"

namespace fcc {
namespace {

constexpr int kMono = 5;  // {1, c3, c1, c2, c1 c3}

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Labels of the orbit of p0 under p -> (g p) mod m: one per distinct cube, the
// first group element reaching it and the wrap floor((g p0) / m).  Returned
// sorted (the class key); cubes[i] is the natural index of label i's cube.
void orbit_labels(const int p0[3], int m, int lg, std::vector<std::array<int, 4>>* labels, std::vector<int>* cubes) {
  const auto& G = weyl_group();
  std::array<std::pair<std::array<int, 4>, int>, 24> found{};
  int cnt = 0;
  for (int w = 0; w < 24; ++w) {
    int q[3], u[3];
    for (int i = 0; i < 3; ++i) {
      q[i] = G[w][3 * i] * p0[0] + G[w][3 * i + 1] * p0[1] + G[w][3 * i + 2] * p0[2];
      u[i] = q[i] >> lg;  // floor division by m = 2^lg
    }
    const int idx = ((((q[0] & (m - 1)) << lg) | (q[1] & (m - 1))) << lg) | (q[2] & (m - 1));
    bool seen = false;
    for (int i = 0; i < cnt; ++i) seen |= found[i].second == idx;
    if (!seen) found[cnt++] = {{w, u[0], u[1], u[2]}, idx};
  }
  std::sort(found.begin(), found.begin() + cnt);
  labels->clear();
  cubes->clear();
  for (int i = 0; i < cnt; ++i) {
    labels->push_back(found[i].first);
    cubes->push_back(found[i].second);
  }
}

std::vector<int> flat_key(const std::vector<std::array<int, 4>>& labels) {
  std::vector<int> k;
  for (const auto& l : labels) k.insert(k.end(), l.begin(), l.end());
  return k;
}

// Templates of one reference node size, read off its derived tables.
struct Family {
  int nl_ref = 0;
  std::vector<double> poly;  // npoly * kMono, constants first
  int npoly = 0, nconst = 0;
  std::vector<OrbitTemplate> templ;
  std::map<std::vector<int>, int> by_key;
};

std::unique_ptr<Family> build_family(int nl) {
  const LevelTables* T = level_tables(nl);
  const GatherBlocks* gb = gather_blocks(nl);
  if (!T || !gb) throw std::bad_alloc();
  const int m = nl / 2, lg = log2i(m);
  // polynomials in the fixed monomial order, keyed by their exact values
  // (every coefficient is a multiple of 1/144)
  auto slot_of = [](int e1, int e2, int e3) {
    if (e1 == 0 && e2 == 0 && e3 == 0) return 0;
    if (e1 == 0 && e2 == 0 && e3 == 1) return 1;
    if (e1 == 1 && e2 == 0 && e3 == 0) return 2;
    if (e1 == 0 && e2 == 1 && e3 == 0) return 3;
    if (e1 == 1 && e2 == 0 && e3 == 1) return 4;
    return -1;
  };
  std::vector<int> mslot(T->nmono);
  for (int q = 0; q < T->nmono; ++q) {
    mslot[q] = slot_of(T->mono[3 * q], T->mono[3 * q + 1], T->mono[3 * q + 2]);
    if (mslot[q] < 0) throw std::runtime_error("unexpected monomial");
  }
  std::map<std::array<long long, kMono>, int> pkey;  // exact key -> first-seen id
  std::vector<std::array<double, kMono>> pval;
  auto poly_id = [&](int pid) {
    std::array<double, kMono> v{};
    for (int q = 0; q < T->nmono; ++q) v[mslot[q]] = T->poly[size_t(pid) * T->nmono + q];
    std::array<long long, kMono> k{};
    for (int q = 0; q < kMono; ++q) k[q] = std::llround(v[q] * 144.0);
    auto it = pkey.find(k);
    if (it != pkey.end()) return it->second;
    const int id = int(pval.size());
    pkey.emplace(k, id);
    pval.push_back(v);
    return id;
  };
  auto fam = std::make_unique<Family>();
  fam->nl_ref = nl;
  std::vector<std::array<int, 4>> labels;
  std::vector<int> cubes;
  std::vector<int> slot_of_cube(size_t(m) * m * m, -1);
  // entries with first-seen polynomial ids; remapped below
  std::vector<std::vector<std::pair<int, int>>> b_rows, c_rows;
  for (int c = 0; c < m * m * m; ++c) {
    if (gb->cube[c] != c) continue;  // not the smallest cube of its block
    const int p0[3] = {c >> (2 * lg), (c >> lg) & (m - 1), c & (m - 1)};
    orbit_labels(p0, m, lg, &labels, &cubes);
    std::vector<int> key = flat_key(labels);
    if (fam->by_key.count(key)) continue;
    const int nc = int(labels.size());
    OrbitTemplate t;
    t.nc = nc;
    t.key = key;
    for (int j = 0; j < nc; ++j) {
      t.w.push_back(labels[j][0]);
      slot_of_cube[cubes[j]] = j;
    }
    // the block of the tables must be this orbit
    for (int q = 0; q < m * m * m; ++q)
      if ((gb->cube[q] == c) != (slot_of_cube[q] >= 0)) throw std::runtime_error("block is not an orbit");
    auto source_slot = [&](uint32_t packed) {
      const int k[3] = {int(packed >> 20), int((packed >> 10) & 1023u), int(packed & 1023u)};
      const int q = ((((k[0] & (m - 1)) << lg) | (k[1] & (m - 1))) << lg) | (k[2] & (m - 1));
      const int o = ((k[0] >> lg) << 2) | ((k[1] >> lg) << 1) | (k[2] >> lg);
      const int j = slot_of_cube[q];
      if (j < 0) throw std::runtime_error("source outside the orbit's octets");
      return j * 8 + o;
    };
    auto cube_slot = [&](uint32_t packed) {  // position def + 2 q
      const int k[3] = {int(packed >> 20), int((packed >> 10) & 1023u), int(packed & 1023u)};
      const int q = (((k[0] >> 1) << lg) | (k[1] >> 1)) << lg | (k[2] >> 1);
      const int f = ((k[0] & 1) << 2) | ((k[1] & 1) << 1) | (k[2] & 1);
      const int j = slot_of_cube[q];
      if (j < 0) throw std::runtime_error("position outside the orbit's cubes");
      return j * 8 + f;
    };
    std::vector<std::vector<std::pair<int, int>>> br(8 * nc), cr(8 * nc);
    for (int j = 0; j < nc; ++j) {
      const int q = cubes[j];
      const int qc[3] = {q >> (2 * lg), (q >> lg) & (m - 1), q & (m - 1)};
      for (int f = 0; f < 8; ++f) {
        // B row (def = f, cube q)
        const int r = q * 8 + f;
        for (int e = T->b_rowptr[r]; e < T->b_rowptr[r + 1]; ++e)
          br[j * 8 + f].push_back({source_slot(T->b_src[e]), poly_id(T->b_pid[e])});
        // C row for the octet point kappa = q + m o (o = f)
        const int kp[3] = {qc[0] + m * ((f >> 2) & 1), qc[1] + m * ((f >> 1) & 1), qc[2] + m * (f & 1)};
        const int rc = ((((kp[0] >> 1) << lg) | (kp[1] >> 1)) << lg | (kp[2] >> 1)) * 8 +
                       (((kp[0] & 1) << 2) | ((kp[1] & 1) << 1) | (kp[2] & 1));
        for (int e = T->c_rowptr[rc]; e < T->c_rowptr[rc + 1]; ++e)
          cr[j * 8 + f].push_back({cube_slot(T->c_src[e]), poly_id(T->c_pid[e])});
      }
    }
    for (int j = 0; j < nc; ++j) slot_of_cube[cubes[j]] = -1;
    fam->by_key.emplace(key, int(fam->templ.size()));
    fam->templ.push_back(std::move(t));
    b_rows.insert(b_rows.end(), br.begin(), br.end());
    c_rows.insert(c_rows.end(), cr.begin(), cr.end());
  }
  // constants first
  const int np = int(pval.size());
  std::vector<int> order(np), newid(np);
  for (int i = 0; i < np; ++i) order[i] = i;
  auto is_const = [&](int i) {
    for (int q = 1; q < kMono; ++q)
      if (pval[i][q] != 0.0) return false;
    return true;
  };
  std::stable_partition(order.begin(), order.end(), is_const);
  fam->npoly = np;
  fam->nconst = 0;
  for (int i = 0; i < np; ++i) fam->nconst += is_const(i) ? 1 : 0;
  if (np > 256) throw std::runtime_error("more than 256 coefficient polynomials");
  fam->poly.resize(size_t(np) * kMono);
  for (int i = 0; i < np; ++i) {
    newid[order[i]] = i;
    for (int q = 0; q < kMono; ++q) fam->poly[size_t(i) * kMono + q] = pval[order[i]][q];
  }
  size_t row = 0;
  for (auto& t : fam->templ) {
    for (int side = 0; side < 2; ++side) {
      std::vector<int>& rp = side == 0 ? t.b_rowptr : t.c_rowptr;
      std::vector<uint16_t>& ent = side == 0 ? t.b_ent : t.c_ent;
      const auto& rows = side == 0 ? b_rows : c_rows;
      rp.assign(1, 0);
      for (int r = 0; r < 8 * t.nc; ++r) {
        for (const auto& e : rows[row + r]) ent.push_back(uint16_t((e.first << 8) | newid[e.second]));
        rp.push_back(int(ent.size()));
      }
    }
    row += size_t(8) * t.nc;
  }
  return fam;
}

const Family* family(int nl_ref) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<Family>> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(nl_ref);
  if (it != cache.end()) return it->second.get();
  try {
    return cache.emplace(nl_ref, build_family(nl_ref)).first->second.get();
  } catch (const std::exception&) {
    return nullptr;
  }
}

uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t k = 0;
  for (int b = 0; b < 10; ++b)
    k |= (uint64_t((x >> b) & 1u) << (3 * b + 2)) | (uint64_t((y >> b) & 1u) << (3 * b + 1)) |
         (uint64_t((z >> b) & 1u) << (3 * b));
  return k;
}

std::unique_ptr<OrbitBlocks> build_blocks(int nl) {
  const Family* fam = family(nl < 16 ? nl : 32);
  if (!fam) return nullptr;
  const int m = nl / 2, lg = log2i(m);
  auto out = std::make_unique<OrbitBlocks>();
  out->nl = nl;
  out->m = m;
  out->npoly = fam->npoly;
  out->nconst = fam->nconst;
  out->poly = fam->poly;
  out->templ = fam->templ;
  out->reps.assign(fam->templ.size(), {});
  // representatives: cubes that are the smallest of their orbit
  const long long cubes = (long long)m * m * m;
  const unsigned nt = std::max(1u, std::min(std::thread::hardware_concurrency(), 64u));
  std::vector<std::vector<std::vector<std::pair<uint64_t, uint32_t>>>> part(
      nt, std::vector<std::vector<std::pair<uint64_t, uint32_t>>>(fam->templ.size()));
  std::atomic<long long> next{0};
  std::atomic<bool> bad{false};
  const auto& G = weyl_group();
  auto work = [&](unsigned t) {
    try {
    std::vector<std::array<int, 4>> labels;
    std::vector<int> cl;
    const long long chunk = 4096;
    for (;;) {
      const long long c0 = next.fetch_add(chunk);
      if (c0 >= cubes || bad.load()) break;
      for (long long c = c0; c < std::min(cubes, c0 + chunk); ++c) {
        const int p[3] = {int(c >> (2 * lg)), int((c >> lg) & (m - 1)), int(c & (m - 1))};
        bool rep = true;
        for (int w = 1; w < 24 && rep; ++w) {
          int q[3];
          for (int i = 0; i < 3; ++i) q[i] = (G[w][3 * i] * p[0] + G[w][3 * i + 1] * p[1] + G[w][3 * i + 2] * p[2]) & (m - 1);
          rep = ((((long long)q[0] << lg) | q[1]) << lg | q[2]) >= c;
        }
        if (!rep) continue;
        orbit_labels(p, m, lg, &labels, &cl);
        auto it = fam->by_key.find(flat_key(labels));
        if (it == fam->by_key.end()) {
          bad.store(true);
          return;
        }
        part[t][it->second].push_back({morton3(p[0], p[1], p[2]), (uint32_t(p[0]) << 20) | (uint32_t(p[1]) << 10) | uint32_t(p[2])});
      }
    }
    } catch (...) {
      bad.store(true);
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back(work, t);
  work(0);
  for (auto& x : th) x.join();
  if (bad.load()) return nullptr;
  for (size_t k = 0; k < fam->templ.size(); ++k) {
    std::vector<std::pair<uint64_t, uint32_t>> all;
    for (unsigned t = 0; t < nt; ++t) all.insert(all.end(), part[t][k].begin(), part[t][k].end());
    std::sort(all.begin(), all.end());
    out->reps[k].reserve(all.size());
    for (const auto& e : all) out->reps[k].push_back(e.second);
  }
  return out;
}

}  // namespace

const OrbitBlocks* orbit_blocks(int nl) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<OrbitBlocks>> cache;
  if (nl < 4 || nl > 1024 || (nl & (nl - 1))) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(nl);
  if (it != cache.end()) return it->second.get();
  try {
    auto b = build_blocks(nl);
    if (!b) return nullptr;
    return cache.emplace(nl, std::move(b)).first->second.get();
  } catch (const std::exception&) {
    return nullptr;
  }
}

}  // namespace fcc
