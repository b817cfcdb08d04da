// C ABI of the SLRF eigensolver.
//
// An engine over pencils.  Each pencil's merged CSR (with its FP32 copy,
// diagonals and sparse-product row order) is validated, built and uploaded once
// and kept in the caller's workspace.  A filter application runs on any set of
// (pencil, L, poles) jobs at once: the batched Krylov kernels serve every
// pole x column of every job in one launch per step.  An outer step of
// Algorithm 1 is one batched filter application followed by Rayleigh-Ritz,
// residuals and the stopping test per pencil.  slrf_ctx is a batch of one
// pencil; slrf_batch keeps a changing set of pencils (continuous batching) in
// one workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <functional>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/slrf.h"
#include "../../include/slrf_testing.h"
#include "dense.h"
#include "kernels.h"

using namespace slrf;

namespace {

constexpr int kRowsPerBlock = 16;   // default rows per row block (4 wavefronts x one row group)
constexpr int kGroup = 4;           // rows of a stencil group (see stencil_groups)
constexpr int kNode = 3;            // rows of a node triple (see node_triples)
constexpr int kRowAlign = 12;       // row-order chunks keep groups and triples whole
constexpr int kRowsPerNodeBlock = 24;  // default rows per block for node-triple pencils
constexpr int kWgPerXcd = 128;      // default workgroups per XCD (grid 8 * 128)
constexpr int kSubBand = 1024;      // default rows per sub-band of the sparse-product row order
constexpr int kTimerSlots = 512;
// largest residual of the previous outer iteration above which the Gram
// products of the first Rayleigh-Ritz projection of the mixed form run on FP32
// MFMA, and the eigenvalue floor of that projection (about the FP32 Gram's
// rounding level relative to its largest eigenvalue)
constexpr double kFirstPassF32Above = 1e-6;
constexpr double kF32GramFloor = 1e-6;
constexpr double kInnerTol32 = 1e-6;  // tightest relative tolerance of an FP32 correction solve
constexpr double kBeyondGammaTarget = 1e-3;  // inner target of the columns beyond gamma
constexpr int kMaxRounds = 6;         // defect-correction rounds per filter application
constexpr int kDefaultPoles = 4;

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Bump allocator over a device region; with base == nullptr it only measures.
struct Carver {
  char* base;
  size_t off = 0, cap = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = al(off + count * sizeof(T));
    return p;
  }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ILU(0) runs one thread per column over all rows: only for narrow patterns.
bool ilu_allowed(int64_t n, int64_t nnz) { return nnz <= 5 * n; }
bool use_ilu_for(int precond, int64_t n, int64_t nnz) {
  return precond == 2 || (precond == 0 && ilu_allowed(n, nnz));
}
bool use_bjac_for(int precond) { return precond == 3; }
// multicolour symmetric Gauss-Seidel (COCG only): block size 1 (precond 4) or 3 (precond 5)
int sgs_block_for(int precond) { return precond == 4 ? 1 : precond == 5 ? 3 : 0; }

// First-fit allocator over a device region (persistent data of a batch).
struct Pool {
  char* base = nullptr;
  std::map<size_t, size_t> free_;  // offset -> size
  void init(char* b, size_t s) {
    base = b;
    free_.clear();
    s &= ~size_t(255);
    if (s) free_[0] = s;
  }
  char* alloc(size_t bytes) {
    bytes = al(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        return base + off;
      }
    }
    return nullptr;
  }
  void release(char* p, size_t bytes) {
    if (!p) return;
    bytes = al(bytes);
    size_t off = (size_t)(p - base);
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + bytes == nx->first) {
      bytes += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == off) {
        off = pv->first;
        bytes += pv->second;
        free_.erase(pv);
      }
    }
    free_[off] = bytes;
  }
};

// ---------------------------------------------------------------------------
// Pencils

// Host copies of a pencil's preconditioner factors for one pole set in one
// Krylov precision (element size rsize), kept across filter applications: the
// poles of a solve do not change between its outer iterations, so the factors
// are computed once per solve and re-uploaded from here.
struct PrecTables {
  int rsize = 0;
  double omega = 1.0;  // SOR relaxation of the SGS factors
  std::vector<double> sigma;
  std::vector<char> ilu, bjac, sgsR, sgsD;
};

struct Pencil {
  int64_t n = 0, nnz = 0;
  int* rowptr = nullptr;
  int* col = nullptr;
  ab_pair<double>* ab64 = nullptr;
  ab_pair<float>* ab32 = nullptr;
  double* diagA = nullptr;
  double* diagB = nullptr;
  float* diagA32 = nullptr;
  float* diagB32 = nullptr;
  int* diagpos = nullptr;
  int* sched = nullptr;
  int* groups = nullptr;  // stencil-group flags (n / kGroup), or null
  int* nodes = nullptr;   // node-triple flags (n / kNode), or null (never both)
  bool use_ilu = false;
  bool use_bjac = false;  // node 3x3 block Jacobi
  // multicolour SGS: block size, colours, nodes by colour, lower / upper coupling CSRs
  int sgs = 0, sgs_ncol = 0;
  int64_t sgs_maxc = 0;  // nodes of the largest colour
  int *sgs_cptr = nullptr, *sgs_nodes = nullptr;
  int *lrp = nullptr, *lcol = nullptr, *urp = nullptr, *ucol = nullptr;
  ab_pair<double>*lab64 = nullptr, *uab64 = nullptr;
  ab_pair<float>*lab32 = nullptr, *uab32 = nullptr;
  int64_t lnnz = 0, unnz = 0;
  char* mem = nullptr;  // device region holding the above
  size_t mem_bytes = 0;
  std::vector<int32_t> h_rp, h_cl, h_dpos;  // host copies for ILU(0) / block Jacobi
  std::vector<double> h_ab;
  mutable PrecTables tables;  // the factors of the last pole set (upload_tables)
};

// The colours of a greedy colouring are at most the largest node degree + 1;
// the colour offsets are sized for kMaxColours.
constexpr int kMaxColours = 1024;

size_t pencil_bytes(int64_t n, int64_t nnz, int precond = 0) {
  const size_t np = (size_t)nnz + kCsrPad;
  size_t b = al((size_t)(n + 1) * 4) + al(np * 4) + al(np * 16) + al(np * 8) + 2 * al((size_t)n * 8) +
             2 * al((size_t)n * 4) + 2 * al((size_t)n * 4) + al((size_t)(n / kGroup + 1) * 4) +
             al((size_t)(n / kNode + 1) * 4);
  if (sgs_block_for(precond)) {
    // colour offsets and nodes; two coupling CSRs (together at most nnz entries)
    b += al((kMaxColours + 1) * 4) + al((size_t)n * 4) + 2 * al((size_t)(n + 1) * 4);
    for (int part = 0; part < 2; ++part) b += al(np * 4) + al(np * 16) + al(np * 8);
  }
  return b;
}

// Greedy colouring of the node graph (block = 1: unknowns; 3: unknowns 3k..3k+2
// form node k): nodes in increasing index, each takes the smallest colour that
// no already coloured neighbour has.  Returns the number of colours.
int greedy_colours(int64_t n, int block, const std::vector<int32_t>& rp, const std::vector<int32_t>& cl,
                   std::vector<int32_t>& colour) {
  const int64_t nodes = n / block;
  colour.assign(nodes, -1);
  std::vector<int64_t> seen(kMaxColours + 1, -1);
  int ncol = 0;
  for (int64_t k = 0; k < nodes; ++k) {
    for (int r = 0; r < block; ++r) {
      const int64_t i = block * k + r;
      for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const int64_t m = cl[q] / block;
        if (m != k && colour[m] >= 0) seen[colour[m]] = k;
      }
    }
    int c = 0;
    while (c < kMaxColours && seen[c] == k) ++c;
    if (c >= kMaxColours) return -1;
    colour[k] = c;
    ncol = std::max(ncol, c + 1);
  }
  return ncol;
}

// Row order of the sparse products.  With upper bandwidth H (max j - i), the
// neighbours of row i lie in [i - H, i + H].  Rows are cut into chunks of H and
// each chunk into S sub-bands of about `band` rows; the order visits sub-band
// s of chunk 0, 1, 2, ... before sub-band s + 1, so consecutive rows in the
// order have overlapping neighbourhoods (for a lexicographic 3D grid: a narrow
// (x, y) band marching along z).  Returns false (natural order) when H is small.
bool band_schedule(int64_t n, const std::vector<int32_t>& rp, const std::vector<int32_t>& cl, int band_rows,
                   std::vector<int32_t>& order) {
  if (band_rows < 0) return false;
  const int64_t target = band_rows > 0 ? band_rows : kSubBand;
  int64_t H = 0;
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] > rp[i]) H = std::max<int64_t>(H, (int64_t)cl[rp[i + 1] - 1] - i);
  if (H <= 2 * target || H >= n) return false;
  H = (H + kRowAlign - 1) / kRowAlign * kRowAlign;  // chunk and sub-band starts keep groups and triples whole
  const int64_t S = (H + target - 1) / target;
  const int64_t band = ((H + S - 1) / S + kRowAlign - 1) / kRowAlign * kRowAlign, nchunk = (n + H - 1) / H;
  order.clear();
  order.reserve(n);
  for (int64_t sb = 0; sb < S; ++sb)
    for (int64_t k = 0; k < nchunk; ++k) {
      const int64_t a = k * H + sb * band, b = std::min({k * H + (sb + 1) * band, (k + 1) * H, n});
      for (int64_t r = a; r < b; ++r) order.push_back((int32_t)r);
    }
  return (int64_t)order.size() == n;
}

// Stencil groups: kGroup consecutive rows i0 .. i0 + 3 (i0 a multiple of kGroup)
// whose entries have the same offsets col - row, in runs of three consecutive
// columns (interior rows of bilinear and trilinear finite-element pencils).  For
// such a group, run j of row r covers columns c_j + r .. c_j + r + 2, so the
// sparse product gathers the six rows c_j .. c_j + 5 once for all four rows.
// Returns one flag per group.
std::vector<int32_t> stencil_groups(int64_t n, const std::vector<int32_t>& rp, const std::vector<int32_t>& cl) {
  const int64_t ng = n / kGroup;
  std::vector<int32_t> g(ng > 0 ? ng : 1, 0);
  for (int64_t q = 0; q < ng; ++q) {
    const int64_t i0 = q * kGroup;
    const int32_t k0 = rp[i0], m = rp[i0 + 1] - rp[i0];
    if (m <= 0 || m % 3 != 0) continue;
    bool ok = true;
    for (int r = 1; r < kGroup && ok; ++r) {
      if (rp[i0 + r + 1] - rp[i0 + r] != m) ok = false;
      for (int32_t k = 0; k < m && ok; ++k)
        if (cl[rp[i0 + r] + k] != cl[k0 + k] + r) ok = false;
    }
    for (int32_t j = 0; j < m && ok; j += 3)
      if (cl[k0 + j + 1] != cl[k0 + j] + 1 || cl[k0 + j + 2] != cl[k0 + j] + 2) ok = false;
    g[q] = ok ? 1 : 0;
  }
  return g;
}

// Node triples: rows 3k, 3k + 1, 3k + 2 with the same column list (the three
// displacement components of a node in vector-valued finite elements: every
// row couples to all components of the same neighbour nodes).  The sparse
// product gathers each column once for the three rows.  Returns one flag per
// triple.
std::vector<int32_t> node_triples(int64_t n, const std::vector<int32_t>& rp, const std::vector<int32_t>& cl) {
  const int64_t nt = n / kNode;
  std::vector<int32_t> g(nt > 0 ? nt : 1, 0);
  for (int64_t q = 0; q < nt; ++q) {
    const int64_t i0 = q * kNode;
    const int32_t k0 = rp[i0], m = rp[i0 + 1] - rp[i0];
    bool ok = m > 0;
    for (int r = 1; r < kNode && ok; ++r) {
      if (rp[i0 + r + 1] - rp[i0 + r] != m) ok = false;
      for (int32_t k = 0; k < m && ok; ++k)
        if (cl[rp[i0 + r] + k] != cl[k0 + k]) ok = false;
    }
    g[q] = ok ? 1 : 0;
  }
  return g;
}

// Validates A and B, merges them into one CSR of (a, b) pairs over the union
// pattern and, with mem != nullptr, uploads it there (pencil_bytes(n, nnz, precond)
// bytes).  With mem == nullptr it only validates and reports nnz of the union.
slrf_status build_pencil(int64_t n, const int32_t* a_rowptr, const int32_t* a_col, const double* a_val,
                         const int32_t* b_rowptr, const int32_t* b_col, const double* b_val, int precond,
                         int band_rows, hipStream_t s, Pencil& P, std::string& err, char* mem,
                         int64_t* nnz_out) {
  if (n < 1 || n > INT32_MAX || !a_rowptr || !a_col || !a_val || !b_rowptr || !b_col || !b_val) {
    err = "bad size or NULL argument";
    return SLRF_E_INVALID_ARG;
  }
  auto check_csr = [&](const int32_t* rp, const int32_t* cl, const double* v, const char* name) -> std::string {
    if (rp[0] != 0) return std::string(name) + ": row_ptr[0] != 0";
    for (int64_t i = 0; i < n; ++i) {
      if (rp[i + 1] < rp[i]) return std::string(name) + ": row_ptr not non-decreasing";
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        if (cl[k] < 0 || cl[k] >= n) return std::string(name) + ": column index out of range";
        if (k > rp[i] && cl[k] <= cl[k - 1]) return std::string(name) + ": columns not strictly increasing";
        if (!std::isfinite(v[k])) return std::string(name) + ": non-finite value";
      }
    }
    return "";
  };
  err = check_csr(a_rowptr, a_col, a_val, "A");
  if (!err.empty()) return SLRF_E_INVALID_ARG;
  err = check_csr(b_rowptr, b_col, b_val, "B");
  if (!err.empty()) return SLRF_E_INVALID_ARG;
  if (precond < 0 || precond > 5) {
    err = "unknown preconditioner";
    return SLRF_E_INVALID_ARG;
  }
  if (precond == 3 && n % 3 != 0) {
    err = "node blocks need three unknowns per node (n divisible by 3)";
    return SLRF_E_INVALID_ARG;
  }
  std::vector<int32_t> rp(n + 1, 0), cl, dpos(n, -1);
  std::vector<double> ab, dA(n, 0.0), dB(n, 0.0);
  cl.reserve(std::max(a_rowptr[n], b_rowptr[n]));
  ab.reserve(2 * (size_t)std::max(a_rowptr[n], b_rowptr[n]));
  for (int64_t i = 0; i < n; ++i) {
    int32_t ka = a_rowptr[i], kb = b_rowptr[i];
    const int32_t ea = a_rowptr[i + 1], eb = b_rowptr[i + 1];
    while (ka < ea || kb < eb) {
      const int32_t ca = ka < ea ? a_col[ka] : INT32_MAX, cb = kb < eb ? b_col[kb] : INT32_MAX;
      const int32_t c = std::min(ca, cb);
      const double va = (ca == c) ? a_val[ka++] : 0.0;
      const double vb = (cb == c) ? b_val[kb++] : 0.0;
      cl.push_back(c);
      ab.push_back(va);
      ab.push_back(vb);
      if (c == i) {
        dA[i] = va;
        dB[i] = vb;
        dpos[i] = (int32_t)cl.size() - 1;
      }
    }
    rp[i + 1] = (int32_t)cl.size();
  }
  for (int64_t i = 0; i < n; ++i)
    if (!(dA[i] > 0) || !(dB[i] > 0)) {
      err = "row " + std::to_string(i) + ": diagonal of A or B not positive";
      return SLRF_E_NOT_SPD;
    }
  const int64_t nnz = (int64_t)cl.size();
  // A and B symmetric (the pencil of Section 1): every stored entry (i, j) of
  // the merged pattern against (j, i), found by bisection in the sorted row j
  // (an entry stored on one side only counts as zero there), to 1e-10 of the
  // diagonal scale sqrt(m_ii m_jj).  Rows are split over host threads; the
  // first failing row is reported.  Checked in the validation pass
  // (mem == nullptr), which both callers run on the same arrays before the pass
  // that uploads.
  if (!mem) {
    constexpr double kSymTol = 1e-10;
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(),
                                                                 nnz / 200000 + 1}));
    std::vector<int64_t> bad(nt, -1), badc(nt, -1);
    auto check_rows = [&](int t) {
      const int64_t i0 = n * t / nt, i1 = n * (t + 1) / nt;
      for (int64_t i = i0; i < i1; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
          const int32_t j = cl[k];
          if (j == i) continue;
          const int32_t* lo = cl.data() + rp[j];
          const int32_t* hi = cl.data() + rp[j + 1];
          const int32_t* f = std::lower_bound(lo, hi, (int32_t)i);
          const bool has = f != hi && *f == i;
          const size_t q = has ? (size_t)(f - cl.data()) : 0;
          const double aji = has ? ab[2 * q] : 0.0, bji = has ? ab[2 * q + 1] : 0.0;
          if (!(std::fabs(ab[2 * (size_t)k] - aji) <= kSymTol * std::sqrt(dA[i] * dA[j])) ||
              !(std::fabs(ab[2 * (size_t)k + 1] - bji) <= kSymTol * std::sqrt(dB[i] * dB[j]))) {
            bad[t] = i;
            badc[t] = j;
            return;
          }
        }
    };
    if (nt == 1) {
      check_rows(0);
    } else {
      std::vector<std::thread> pool;
      for (int t = 0; t < nt; ++t) pool.emplace_back(check_rows, t);
      for (auto& th : pool) th.join();
    }
    for (int t = 0; t < nt; ++t)
      if (bad[t] >= 0) {
        const int64_t i = bad[t], j = badc[t];
        const int32_t* f = std::lower_bound(cl.data() + rp[i], cl.data() + rp[i + 1], (int32_t)j);
        const size_t k = (size_t)(f - cl.data());
        const int32_t* g = std::lower_bound(cl.data() + rp[j], cl.data() + rp[j + 1], (int32_t)i);
        const bool has = g != cl.data() + rp[j + 1] && *g == i;
        const double aji = has ? ab[2 * (size_t)(g - cl.data())] : 0.0;
        const bool a_bad = !(std::fabs(ab[2 * k] - aji) <= kSymTol * std::sqrt(dA[i] * dA[j]));
        err = std::string(a_bad ? "A" : "B") + " is not symmetric: entries (" + std::to_string(i) + ", " +
              std::to_string(j) + ") and (" + std::to_string(j) + ", " + std::to_string(i) + ") differ";
        return SLRF_E_INVALID_ARG;
      }
  }
  if (nnz_out) *nnz_out = nnz;
  if (precond == 2 && !ilu_allowed(n, nnz)) {
    err = "ILU(0) needs a narrow pattern (nnz <= 5 n)";
    return SLRF_E_INVALID_ARG;
  }
  if (!mem) return SLRF_OK;
  P.n = n;
  P.nnz = nnz;
  P.use_ilu = use_ilu_for(precond, n, nnz);
  P.use_bjac = use_bjac_for(precond);
  const std::vector<int32_t> groups = stencil_groups(n, rp, cl), nodes = node_triples(n, rp, cl);
  int64_t n_group = 0, n_node = 0;
  for (int32_t f : groups) n_group += f != 0;
  for (int32_t f : nodes) n_node += f != 0;
  // multicolour SGS: precond 5 takes the 3 x 3 node blocks where the pencil is
  // made of nodes (n divisible by 3, at least half of its rows in node triples)
  // and the point form elsewhere, so that one batch serves both kinds
  P.sgs = sgs_block_for(precond);
  if (P.sgs == 3 && !(n % 3 == 0 && 2 * kNode * n_node >= n)) P.sgs = 1;
  P.mem = mem;
  P.mem_bytes = pencil_bytes(n, nnz, precond);
  Carver cv{mem, 0, P.mem_bytes};
  P.rowptr = cv.take<int>(n + 1);
  P.col = cv.take<int>(nnz + kCsrPad);
  P.ab64 = cv.take<ab_pair<double>>(nnz + kCsrPad);
  P.ab32 = cv.take<ab_pair<float>>(nnz + kCsrPad);
  P.diagA = cv.take<double>(n);
  P.diagB = cv.take<double>(n);
  P.diagA32 = cv.take<float>(n);
  P.diagB32 = cv.take<float>(n);
  P.diagpos = cv.take<int>(n);
  int* sched_dev = cv.take<int>(n);
  int* groups_dev = cv.take<int>(n / kGroup + 1);
  int* nodes_dev = cv.take<int>(n / kNode + 1);
  // multicolour SGS tables: colours of the nodes, nodes by colour, and the merged
  // CSR split into couplings to lower and to higher colours (same-node entries
  // form the diagonal blocks and belong to neither)
  std::vector<int32_t> cptr, cnodes, lrp, lcl, urp, ucl;
  std::vector<double> lab, uab;
  if (P.sgs) {
    const int bs = P.sgs;
    std::vector<int32_t> colour;
    const int ncol = greedy_colours(n, bs, rp, cl, colour);
    if (ncol < 1) {
      err = "node graph needs more than " + std::to_string(kMaxColours) + " colours";
      return SLRF_E_INVALID_ARG;
    }
    P.sgs_ncol = ncol;
    const int64_t nodes = n / bs;
    cptr.assign(ncol + 1, 0);
    for (int64_t k = 0; k < nodes; ++k) cptr[colour[k] + 1]++;
    for (int c = 0; c < ncol; ++c) cptr[c + 1] += cptr[c];
    cnodes.resize(nodes);
    std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t k = 0; k < nodes; ++k) cnodes[fill[colour[k]]++] = (int32_t)k;
    P.sgs_maxc = 1;
    for (int c = 0; c < ncol; ++c) P.sgs_maxc = std::max<int64_t>(P.sgs_maxc, cptr[c + 1] - cptr[c]);
    lrp.assign(n + 1, 0);
    urp.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
      const int ci = colour[i / bs];
      for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const int cj = colour[cl[q] / bs];
        if (cj < ci) {
          lcl.push_back(cl[q]);
          lab.push_back(ab[2 * (size_t)q]);
          lab.push_back(ab[2 * (size_t)q + 1]);
        } else if (cj > ci) {
          ucl.push_back(cl[q]);
          uab.push_back(ab[2 * (size_t)q]);
          uab.push_back(ab[2 * (size_t)q + 1]);
        } else if (cl[q] / bs != i / bs) {
          err = "colouring left two coupled nodes alike";
          return SLRF_E_INVALID_ARG;
        }
      }
      lrp[i + 1] = (int32_t)lcl.size();
      urp[i + 1] = (int32_t)ucl.size();
    }
    P.lnnz = (int64_t)lcl.size();
    P.unnz = (int64_t)ucl.size();
    P.sgs_cptr = cv.take<int>(kMaxColours + 1);
    P.sgs_nodes = cv.take<int>(n);
    P.lrp = cv.take<int>(n + 1);
    P.urp = cv.take<int>(n + 1);
    P.lcol = cv.take<int>(nnz + kCsrPad);
    P.lab64 = cv.take<ab_pair<double>>(nnz + kCsrPad);
    P.lab32 = cv.take<ab_pair<float>>(nnz + kCsrPad);
    P.ucol = cv.take<int>(nnz + kCsrPad);
    P.uab64 = cv.take<ab_pair<double>>(nnz + kCsrPad);
    P.uab32 = cv.take<ab_pair<float>>(nnz + kCsrPad);
    // kCsrPad zero entries after each part (whole-chunk reads)
    lcl.resize(lcl.size() + kCsrPad, 0);
    ucl.resize(ucl.size() + kCsrPad, 0);
    lab.resize(2 * lcl.size(), 0.0);
    uab.resize(2 * ucl.size(), 0.0);
  }
  std::vector<int32_t> order;
  P.sched = band_schedule(n, rp, cl, band_rows, order) ? sched_dev : nullptr;
  // one kind per pencil: the one that covers more rows
  P.nodes = n_node > 0 && kNode * n_node >= kGroup * n_group ? nodes_dev : nullptr;
  P.groups = n_group > 0 && !P.nodes ? groups_dev : nullptr;
  // kCsrPad zero entries (column 0, coefficients 0) after the last entry
  cl.resize(nnz + kCsrPad, 0);
  ab.resize(2 * (size_t)(nnz + kCsrPad), 0.0);
  std::vector<float> ab32(2 * (size_t)(nnz + kCsrPad)), dA32(n), dB32(n);
  for (size_t k = 0; k < ab32.size(); ++k) ab32[k] = (float)ab[k];
  for (int64_t i = 0; i < n; ++i) {
    dA32[i] = (float)dA[i];
    dB32[i] = (float)dB[i];
  }
  auto cp = [&](void* dst, const void* src, size_t b) { return hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, s); };
  const size_t np = (size_t)nnz + kCsrPad;
  if (cp(P.rowptr, rp.data(), 4 * (n + 1)) != hipSuccess || cp(P.col, cl.data(), 4 * np) != hipSuccess ||
      cp(P.ab64, ab.data(), 16 * np) != hipSuccess || cp(P.ab32, ab32.data(), 8 * np) != hipSuccess ||
      cp(P.diagA, dA.data(), 8 * n) != hipSuccess || cp(P.diagB, dB.data(), 8 * n) != hipSuccess ||
      cp(P.diagA32, dA32.data(), 4 * n) != hipSuccess || cp(P.diagB32, dB32.data(), 4 * n) != hipSuccess ||
      cp(P.diagpos, dpos.data(), 4 * n) != hipSuccess ||
      (P.sched && cp(P.sched, order.data(), 4 * n) != hipSuccess) ||
      (P.groups && cp(P.groups, groups.data(), 4 * groups.size()) != hipSuccess) ||
      (P.nodes && cp(P.nodes, nodes.data(), 4 * nodes.size()) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess) {
    err = "upload of the merged CSR failed";
    return SLRF_E_DEVICE;
  }
  if (P.sgs) {
    std::vector<float> lab32(lab.size()), uab32(uab.size());
    for (size_t k = 0; k < lab.size(); ++k) lab32[k] = (float)lab[k];
    for (size_t k = 0; k < uab.size(); ++k) uab32[k] = (float)uab[k];
    if (cp(P.sgs_cptr, cptr.data(), 4 * cptr.size()) != hipSuccess ||
        cp(P.sgs_nodes, cnodes.data(), 4 * cnodes.size()) != hipSuccess ||
        cp(P.lrp, lrp.data(), 4 * lrp.size()) != hipSuccess || cp(P.urp, urp.data(), 4 * urp.size()) != hipSuccess ||
        cp(P.lcol, lcl.data(), 4 * lcl.size()) != hipSuccess || cp(P.ucol, ucl.data(), 4 * ucl.size()) != hipSuccess ||
        cp(P.lab64, lab.data(), 8 * lab.size()) != hipSuccess || cp(P.uab64, uab.data(), 8 * uab.size()) != hipSuccess ||
        cp(P.lab32, lab32.data(), 4 * lab32.size()) != hipSuccess ||
        cp(P.uab32, uab32.data(), 4 * uab32.size()) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      err = "upload of the colour tables failed";
      return SLRF_E_DEVICE;
    }
  }
  if (P.use_ilu || P.use_bjac || P.sgs) {
    P.h_rp = std::move(rp);
    P.h_cl = std::move(cl);
    P.h_ab = std::move(ab);
    P.h_dpos = std::move(dpos);
  }
  return SLRF_OK;
}

// ILU(0) of A - sigma B on the merged pattern (row-wise IKJ elimination without
// fill); the U diagonal is returned inverted.
bool ilu0_factor(const Pencil& P, std::complex<double> sigma, std::vector<std::complex<double>>& f) {
  const int64_t n = P.n, nnz = P.nnz;
  const auto& rp = P.h_rp;
  const auto& cl = P.h_cl;
  const auto& dp = P.h_dpos;
  f.resize(nnz);
  for (int64_t k = 0; k < nnz; ++k) f[k] = std::complex<double>(P.h_ab[2 * k], 0.0) - sigma * P.h_ab[2 * k + 1];
  for (int64_t i = 0; i < n; ++i) {
    for (int32_t k = rp[i]; k < dp[i]; ++k) {
      const int32_t c = cl[k];
      f[k] /= f[dp[c]];
      const std::complex<double> lik = f[k];
      int32_t a = k + 1, b = dp[c] + 1;
      while (a < rp[i + 1] && b < rp[c + 1]) {
        if (cl[a] == cl[b]) {
          f[a] -= lik * f[b];
          ++a;
          ++b;
        } else if (cl[a] < cl[b]) {
          ++a;
        } else {
          ++b;
        }
      }
    }
    if (std::abs(f[dp[i]]) == 0.0 || !std::isfinite(std::abs(f[dp[i]]))) return false;
  }
  for (int64_t i = 0; i < n; ++i) f[dp[i]] = 1.0 / f[dp[i]];
  return true;
}

// Inverted 3x3 node blocks of A - sigma B (node k: unknowns 3k..3k+2), row-major,
// by Gauss-Jordan elimination with partial pivoting.  False if a block is singular.
bool bjac3_factor(const Pencil& P, std::complex<double> sigma, std::vector<std::complex<double>>& f) {
  using C = std::complex<double>;
  const int64_t nodes = P.n / 3;
  f.assign(nodes * 9, C(0.0));
  for (int64_t k = 0; k < nodes; ++k) {
    C m[3][6] = {};
    for (int r = 0; r < 3; ++r) {
      const int64_t i = 3 * k + r;
      for (int32_t q = P.h_rp[i]; q < P.h_rp[i + 1]; ++q) {
        const int64_t c = P.h_cl[q] - 3 * k;
        if (c >= 0 && c < 3) m[r][c] = C(P.h_ab[2 * q], 0.0) - sigma * P.h_ab[2 * q + 1];
      }
      m[r][3 + r] = 1.0;
    }
    for (int col = 0; col < 3; ++col) {
      int piv = col;
      for (int r = col + 1; r < 3; ++r)
        if (std::abs(m[r][col]) > std::abs(m[piv][col])) piv = r;
      if (!(std::abs(m[piv][col]) > 0.0) || !std::isfinite(std::abs(m[piv][col]))) return false;
      if (piv != col)
        for (int q = 0; q < 6; ++q) std::swap(m[piv][q], m[col][q]);
      const C inv = 1.0 / m[col][col];
      for (int q = 0; q < 6; ++q) m[col][q] *= inv;
      for (int r = 0; r < 3; ++r)
        if (r != col) {
          const C fr = m[r][col];
          for (int q = 0; q < 6; ++q) m[r][q] -= fr * m[col][q];
        }
    }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) f[k * 9 + 3 * r + c] = m[r][3 + c];
  }
  return true;
}

double merged_csr_bytes(const Pencil& P, size_t value_bytes) {
  return (double)(P.n + 1) * 4 + (double)P.nnz * (4 + value_bytes);
}

// ---------------------------------------------------------------------------
// Pole design (cached per (N, alpha, beta) at gamma = 1)

std::mutex g_design_mu;
std::map<std::tuple<int, double, double>, std::vector<double>> g_design_cache;

bool design_unit_cached(int N, double alpha, double beta, std::vector<double>& out /* 3N */) {
  std::lock_guard<std::mutex> lk(g_design_mu);
  auto key = std::make_tuple(N, alpha, beta);
  auto it = g_design_cache.find(key);
  if (it != g_design_cache.end()) {
    out = it->second;
    return true;
  }
  std::vector<double> xi(N), om(2 * N);
  if (!design_poles_unit(N, alpha, beta, xi.data(), om.data())) return false;
  out.assign(3 * N, 0.0);
  for (int j = 0; j < N; ++j) {
    out[j] = xi[j];
    out[N + 2 * j] = om[2 * j];
    out[N + 2 * j + 1] = om[2 * j + 1];
  }
  g_design_cache[key] = out;
  return true;
}

// ---------------------------------------------------------------------------
// Engine state shared by contexts and batches

struct Env {
  hipStream_t stream = nullptr;
  slrf_options opt{};
  bool verbose = false;
  std::string err;
  LaunchTimer timer;
  std::vector<hipEvent_t> events;
  ~Env() {
    for (hipEvent_t e : events)
      if (e) (void)hipEventDestroy(e);
  }
  bool setup_timer(int* d_counts) {
    timer.d_counts = d_counts;
    if (!opt.profile) return true;
    events.assign(2 * kTimerSlots, nullptr);
    for (auto& e : events)
      if (hipEventCreate(&e) != hipSuccess) return false;
    timer.events = events.data();
    timer.capacity = kTimerSlots;
    launch_fill_zero(stream, d_counts, 4 * kTimerSlots);
    return hipStreamSynchronize(stream) == hipSuccess;
  }
};

slrf_status fail(Env& env, slrf_status s, const std::string& msg) {
  env.err = msg;
  return s;
}

#define HIPCHK(env, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(env, SLRF_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

slrf_status setup_env(Env& env, const slrf_options* opt, void* hip_stream) {
  if (opt)
    env.opt = *opt;
  else
    slrf_default_options(&env.opt);
  env.verbose = getenv("SLRF_VERBOSE") != nullptr;
  env.stream = (hipStream_t)hip_stream;
  if (env.opt.precision != SLRF_FP64 && env.opt.precision != SLRF_MIXED)
    return fail(env, SLRF_E_INVALID_ARG, "unknown precision");
  if (env.opt.precond < 0 || env.opt.precond > 5) return fail(env, SLRF_E_INVALID_ARG, "unknown preconditioner");
  if (sgs_block_for(env.opt.precond) && env.opt.solver != 1)
    return fail(env, SLRF_E_INVALID_ARG, "the multicolour SGS preconditioner runs with COCG only (solver = 1)");
  if (env.opt.solver != 0 && env.opt.solver != 1) return fail(env, SLRF_E_INVALID_ARG, "unknown inner solver");
  if (env.opt.recycle != 0 && env.opt.recycle != 1) return fail(env, SLRF_E_INVALID_ARG, "recycle must be 0 or 1");
  if (env.opt.sgs_omega != 0.0 && !(env.opt.sgs_omega > 0.0 && env.opt.sgs_omega < 2.0))
    return fail(env, SLRF_E_INVALID_ARG, "sgs_omega must be 0 (by block size) or lie in (0, 2)");
  if (env.opt.solver == 1) {
    // COCG needs a complex-symmetric preconditioner: point or node block Jacobi,
    // or the multicolour SGS
    if (env.opt.precond == 2)
      return fail(env, SLRF_E_INVALID_ARG,
                  "COCG takes point or node block Jacobi or the multicolour SGS (ILU(0) is not symmetric)");
    if (env.opt.precond == 0) env.opt.precond = 1;
  }
  if (!(env.opt.inner_tol >= 0) || !(env.opt.outer_tol >= 0))
    return fail(env, SLRF_E_INVALID_ARG, "tolerances must be non-negative");
  if (env.opt.tile_rows < 0 || env.opt.tile_rows > 64 || env.opt.tile_wgs < 0 ||
      env.opt.tile_wgs * 8 > kMaxGrid || env.opt.band_rows < -1)
    return fail(env, SLRF_E_INVALID_ARG, "tile_rows must be in [0, 64], tile_wgs in [0, 256], band_rows >= -1");
  return SLRF_OK;
}

// SOR relaxation factor of a pencil's multicolour SGS: the option, or by block
// size when it is 0.  Under-relaxed node blocks take fewer iterations on the
// 48^3 elasticity pencil (complete solve 41.3 s at 1, 35.6 s at 0.65 .. 0.8,
// 45.5 s at 1.2), while the 64^3 scalar pencil's point sweeps are fastest at 1
// (3.05 s; 3.25 s at 0.85, 3.50 s at 0.7).
constexpr double kSgsOmegaNode = 0.7;
double sgs_omega_of(const Env& env, const Pencil& P) {
  if (env.opt.sgs_omega > 0.0) return env.opt.sgs_omega;
  return P.sgs == 3 ? kSgsOmegaNode : 1.0;
}

// The point SGS takes its D and D^{-1} from the Jacobi diagonals: with the SOR
// relaxation they hold (2 / omega - 1) d (what the split form subtracts) and
// omega / d (the inverse of d / omega); no other kernel reads them for such a
// pencil.
double point_sgs_cd(const Env& env, const Pencil& P) { return P.sgs == 1 ? 2.0 / sgs_omega_of(env, P) - 1.0 : 1.0; }
double point_sgs_ci(const Env& env, const Pencil& P) { return P.sgs == 1 ? sgs_omega_of(env, P) : 1.0; }

// Reads back the event pairs and tile counters of the current window into the
// kernel statistics, then clears the window.
slrf_status harvest_timer(Env& env, int G, int64_t n_tiles, int64_t total_cols, slrf_filter_stats* fs) {
  LaunchTimer& tm = env.timer;
  if (tm.used == 0) return SLRF_OK;
  std::vector<int> cnt(tm.used);
  HIPCHK(env, hipMemcpyAsync(cnt.data(), tm.d_counts, 4 * (size_t)tm.used, hipMemcpyDeviceToHost, env.stream));
  HIPCHK(env, hipStreamSynchronize(env.stream));
  for (int u = 0; u < tm.used; ++u) {
    float ms = 0;
    HIPCHK(env, hipEventElapsedTime(&ms, tm.events[2 * u], tm.events[2 * u + 1]));
    const LaunchTimer::Rec& r = tm.recs[u];
    // the counter adds one per (workgroup, tile) processed
    const double total_tiles = (double)(r.grid > 0 ? r.grid : G) * (double)n_tiles;
    const double bytes = r.tile_bytes * (double)cnt[u] / total_tiles + (cnt[u] > 0 ? r.fixed : 0.0);
    if (r.kind == 0) {
      fs->spmm_seconds += 1e-3 * ms;
      fs->spmm_launches += 1;
      fs->spmm_bytes += bytes;
      fs->spmm_columns += r.share * (double)total_cols * (double)cnt[u] / (double)total_tiles;
    } else {
      fs->update_seconds += 1e-3 * ms;
      fs->update_launches += 1;
      fs->update_bytes += bytes;
    }
  }
  tm.used = 0;
  launch_fill_zero(env.stream, tm.d_counts, 4 * (size_t)tm.capacity);
  return SLRF_OK;
}

slrf_status check_poles(Env& env, const slrf_poles* p, int max_N) {
  if (!p || p->n_poles < 1 || !p->sigma || !p->weight)
    return fail(env, SLRF_E_INVALID_ARG, "pole set is NULL or empty");
  if (p->n_poles > max_N) return fail(env, SLRF_E_INVALID_ARG, "more poles than the workspace was sized for");
  for (int j = 0; j < p->n_poles; ++j) {
    const double a = p->sigma[2 * j], b = p->sigma[2 * j + 1], c = p->weight[2 * j], d = p->weight[2 * j + 1];
    if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c) || !std::isfinite(d))
      return fail(env, SLRF_E_INVALID_ARG, "non-finite pole or weight");
    if (!(b > 0)) return fail(env, SLRF_E_INVALID_ARG, "poles must lie in the upper half plane (Im sigma > 0)");
  }
  return SLRF_OK;
}

// Node blocks D_k of A - sigma B (row-major) and their complex-symmetric factors
// R_k, lower triangular with D_k = R_k R_k^T (no conjugation: D_k is complex
// symmetric), by the Cholesky recurrences with complex square roots.  False if
// a pivot vanishes.
bool sgs3_factor(const Pencil& P, std::complex<double> sigma, std::vector<std::complex<double>>& Rf,
                 std::vector<std::complex<double>>& Df) {
  using C = std::complex<double>;
  const int64_t nodes = P.n / 3;
  Rf.assign(nodes * 9, C(0.0));
  Df.assign(nodes * 9, C(0.0));
  for (int64_t k = 0; k < nodes; ++k) {
    C* d = &Df[9 * k];
    for (int r = 0; r < 3; ++r) {
      const int64_t i = 3 * k + r;
      for (int32_t q = P.h_rp[i]; q < P.h_rp[i + 1]; ++q) {
        const int64_t c = P.h_cl[q] - 3 * k;
        if (c >= 0 && c < 3) d[3 * r + c] = C(P.h_ab[2 * q], 0.0) - sigma * P.h_ab[2 * q + 1];
      }
    }
    C* R = &Rf[9 * k];
    for (int j = 0; j < 3; ++j) {
      C piv = d[3 * j + j];
      for (int m = 0; m < j; ++m) piv -= R[3 * j + m] * R[3 * j + m];
      const C rjj = std::sqrt(piv);
      if (!(std::abs(rjj) > 0.0) || !std::isfinite(std::abs(rjj))) return false;
      R[3 * j + j] = rjj;
      for (int i = j + 1; i < 3; ++i) {
        C v = d[3 * i + j];
        for (int m = 0; m < j; ++m) v -= R[3 * i + m] * R[3 * j + m];
        R[3 * i + j] = v / rjj;
      }
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// Batched filter application

struct FilterJob {
  const Pencil* P;
  int L, N;
  const double* sigma;   // host, 2N
  const double* weight;  // host, 2N
  const double* X;       // device (n, L)
  double* U;             // device (n, L)
  double target;         // relative accuracy of the shifted solves
  const double* rhs_target = nullptr;  // mixed precision: per right-hand side (L), or null (target)
  slrf_filter_stats stats;
  // warm start (mixed precision): scratch for C = X_prev^T B X_new
  double* gpart = nullptr;  // gram_chunks(n, L) * 2 * L * L
  double* C = nullptr;      // L * L
  double* Cb = nullptr;     // L * L
  int nch = 0;
  // element offsets of the job's (n, Kp) blocks and (n, L) real blocks in the
  // layout (set by place_jobs)
  int64_t blk = 0, rl = 0;
  // warm starts (mixed precision): the pencil's copies of the previous
  // application's Y and B X (null: not kept), and whether they are valid
  cx<double>* yprev = nullptr;
  double* fprev = nullptr;
  bool warm = false;
};

struct JobShape {
  int64_t n, nnz;
  int L, N;
  bool ilu;              // ILU(0) factors of this pencil
  bool general = false;  // count the p and s blocks even without another preconditioner (bounds)
  bool bjac = false;     // node block-Jacobi inverses of this pencil
  int sgs = 0;           // multicolour SGS block size of this pencil (its R, D and D^{-1})
};

// Device layout of one batched filter application.  Carving with a null base
// measures it; partial sums are sized for kMaxGrid workgroups so the size does
// not depend on the grid a batch picks.
struct FilterLayout {
  int64_t EB = 0, ER = 0, ED = 0, Ktot = 0, n_tiles = 0, ilu_vals = 0, bjac_vals = 0, sgs_vals = 0;
  bool any_ilu = false, any_bjac = false;
  int sgs = 0;  // block size of the batch's multicolour SGS (all its pencils share the option)
  void* vec[9] = {};  // x r ph v sh t [p s] [complex shadow residual]
  double* rhat = nullptr;
  void* d = nullptr;
  void* dinv = nullptr;
  void* sigma_col = nullptr;
  cx<double>* sigma_col64 = nullptr;
  cx<double>* Y = nullptr;
  cx<double>* R = nullptr;
  double* F = nullptr;
  double* w = nullptr;
  void* sig_j = nullptr;
  void* part_a = nullptr;
  void* part_b = nullptr;
  double* part64 = nullptr;
  void* scal[4] = {};  // rho alpha omega beta
  void* fnorm = nullptr;
  void* rnorm = nullptr;
  int* flags = nullptr;
  int* iters = nullptr;
  double* fnorm64 = nullptr;
  double* scale = nullptr;
  double* relres = nullptr;
  double* tol64 = nullptr;
  float* tol32 = nullptr;
  int* count = nullptr;
  int* active = nullptr;
  int* n_active = nullptr;
  Inst* inst = nullptr;
  int* tile_inst = nullptr;
  int* col_inst = nullptr;
  void* ilu = nullptr;
  void* bjac = nullptr;
  void* sgsR = nullptr;  // multicolour SGS: R (point: ED values; blocks: sgs_vals)
  void* sgsD = nullptr;  // and the node blocks D (blocks only)
  int precs() const { return (any_ilu ? 1 : 0) | (any_bjac ? 2 : 0); }
};

// Columns per lane of the Krylov kernels: 2 adjacent complex FP32 values or one
// complex FP64 value (16 B either way); a tile is W = 64 lanes wide (128 FP32 or
// 64 FP64 columns, 1 KB per row).  A pencil's K columns are padded to Kp, a
// multiple of W, and its blocks are stored tile-major: tile t is a contiguous
// n x W panel, so a tile's rows are 1 KB apart for any K (the vector updates
// stream about 3% faster than over a row-major (n, Kp) block).  The mixed
// form's FP64 blocks use the FP32 tiles (two complex FP64 values per lane).
int lane_width(bool mixed) { return mixed ? 2 : 1; }
int tile_width(bool mixed) { return 64 * lane_width(mixed); }
int64_t padded_k(int64_t K, bool mixed) {
  const int64_t W = tile_width(mixed);
  return (K + W - 1) / W * W;
}

// Block offsets of the jobs: one after the other in the layout.
void place_jobs(std::vector<FilterJob>& jobs, bool mixed) {
  int64_t blk = 0, rl = 0;
  for (auto& j : jobs) {
    j.blk = blk;
    j.rl = rl;
    blk += j.P->n * padded_k((int64_t)j.N * j.L, mixed);
    rl += j.P->n * j.L;
  }
}

// Sizes of a set of jobs: the block, real-block and diagonal-block elements,
// padded columns and tiles, and which preconditioner tables the set needs.
void shape_totals(const std::vector<JobShape>& js, bool mixed, FilterLayout& lo, int64_t& sumN,
                  bool& any_general) {
  lo.EB = lo.ER = lo.ED = lo.Ktot = lo.n_tiles = lo.ilu_vals = lo.bjac_vals = lo.sgs_vals = 0;
  lo.any_ilu = lo.any_bjac = false;
  lo.sgs = 0;
  sumN = 0;
  any_general = false;
  const int V = lane_width(mixed);
  for (const auto& j : js) {
    const int64_t Kp = padded_k((int64_t)j.N * j.L, mixed);
    lo.EB += j.n * Kp;
    lo.ER += j.n * j.L;
    lo.ED += j.n * j.N;
    lo.Ktot += Kp;
    lo.n_tiles += (Kp + 64 * V - 1) / (64 * V);
    sumN += j.N;
    if (j.ilu) {
      lo.any_ilu = true;
      lo.ilu_vals += (int64_t)j.N * j.nnz;
    }
    if (j.bjac || j.sgs == 3) {
      lo.any_bjac = lo.any_bjac || j.bjac;
      lo.bjac_vals += (int64_t)j.N * (j.n / 3) * 9;
    }
    if (j.sgs) {
      lo.sgs = std::max(lo.sgs, j.sgs);
      lo.sgs_vals += j.sgs == 3 ? (int64_t)j.N * (j.n / 3) * 9 : (int64_t)j.n * j.N;
    }
    if (j.general) any_general = true;
  }
}

void carve_filter(Carver& cv, const std::vector<JobShape>& js, bool mixed, FilterLayout& lo) {
  lo = FilterLayout{};
  int64_t sumN = 0;
  bool any_general = false;
  shape_totals(js, mixed, lo, sumN, any_general);
  const size_t cs = mixed ? 8 : 16;  // complex size in the Krylov precision
  const size_t rs = cs / 2;
  // with any ILU(0) or block-Jacobi pencil in the batch, every pencil keeps p and s
  const int nvec = 6 + (lo.any_ilu || lo.any_bjac || any_general ? 2 : 0);
  for (int v = 0; v < nvec; ++v) lo.vec[v] = cv.take<char>((size_t)lo.EB * cs);
  if (mixed) {
    lo.vec[8] = cv.take<char>((size_t)lo.EB * cs);
    lo.Y = cv.take<cx<double>>(lo.EB);
    lo.R = cv.take<cx<double>>(lo.EB);
    lo.F = cv.take<double>(lo.ER);
    lo.sigma_col64 = cv.take<cx<double>>(lo.Ktot);
    lo.part64 = cv.take<double>((size_t)kMaxGrid * lo.Ktot);
    lo.fnorm64 = cv.take<double>(lo.Ktot);
    lo.scale = cv.take<double>(lo.Ktot);
    lo.relres = cv.take<double>(lo.Ktot);
    lo.tol64 = cv.take<double>(lo.Ktot);
    lo.tol32 = cv.take<float>(lo.Ktot);
  } else {
    lo.rhat = cv.take<double>(lo.ER);
  }
  lo.d = cv.take<char>((size_t)lo.ED * cs);
  lo.dinv = cv.take<char>((size_t)lo.ED * cs);
  lo.sigma_col = cv.take<char>((size_t)lo.Ktot * cs);
  lo.sig_j = cv.take<char>((size_t)sumN * cs);
  lo.w = cv.take<double>(2 * sumN);
  lo.part_a = cv.take<char>((size_t)kMaxGrid * lo.Ktot * cs);
  lo.part_b = cv.take<char>((size_t)kMaxGrid * lo.Ktot * rs);
  for (int q = 0; q < 4; ++q) lo.scal[q] = cv.take<char>((size_t)lo.Ktot * cs);
  lo.fnorm = cv.take<char>((size_t)lo.Ktot * rs);
  lo.rnorm = cv.take<char>((size_t)lo.Ktot * rs);
  lo.flags = cv.take<int>(lo.Ktot);
  lo.iters = cv.take<int>(lo.Ktot);
  lo.count = cv.take<int>(64);
  lo.active = cv.take<int>(lo.n_tiles);
  lo.n_active = cv.take<int>(64);
  lo.inst = cv.take<Inst>(js.size());
  lo.tile_inst = cv.take<int>(lo.n_tiles);
  lo.col_inst = cv.take<int>(lo.Ktot);
  if (lo.any_ilu) lo.ilu = cv.take<char>((size_t)lo.ilu_vals * cs);
  if (lo.bjac_vals) lo.bjac = cv.take<char>((size_t)lo.bjac_vals * cs);
  if (lo.sgs) {
    lo.sgsR = cv.take<char>((size_t)lo.sgs_vals * cs);
    if (lo.sgs == 3) lo.sgsD = cv.take<char>((size_t)lo.sgs_vals * cs);
  }
}

size_t filter_arena_bytes(const std::vector<JobShape>& js, bool mixed) {
  Carver cv{nullptr, 0, 0};
  FilterLayout lo;
  carve_filter(cv, js, mixed, lo);
  return cv.off;
}

template <typename R>
KrylovState<R> make_state(const FilterLayout& lo) {
  KrylovState<R> st{};
  st.x = (cx<R>*)lo.vec[0];
  st.r = (cx<R>*)lo.vec[1];
  st.ph = (cx<R>*)lo.vec[2];
  st.v = (cx<R>*)lo.vec[3];
  st.sh = (cx<R>*)lo.vec[4];
  st.t = (cx<R>*)lo.vec[5];
  st.p = (cx<R>*)lo.vec[6];
  st.s = (cx<R>*)lo.vec[7];
  st.rhat = std::is_same<R, double>::value ? (const R*)lo.rhat : nullptr;
  st.rhat_cx = (const cx<R>*)lo.vec[8];
  st.d = (const cx<R>*)lo.d;
  st.dinv = (const cx<R>*)lo.dinv;
  st.sigma_col = (const cx<R>*)lo.sigma_col;
  st.part_a = (cx<R>*)lo.part_a;
  st.part_b = (R*)lo.part_b;
  st.rho = (cx<R>*)lo.scal[0];
  st.alpha = (cx<R>*)lo.scal[1];
  st.omega = (cx<R>*)lo.scal[2];
  st.beta = (cx<R>*)lo.scal[3];
  st.fnorm = (R*)lo.fnorm;
  st.rnorm = (R*)lo.rnorm;
  st.flags = lo.flags;
  st.iters = lo.iters;
  return st;
}

struct Tiling {
  int rpb, wgs;  // rows per row block, workgroups per XCD
};

// Default rows per block: 16 (four stencil groups per workgroup), or 24 (two
// node triples per wavefront) when the batch's pencils have node triples and no
// stencil groups.
Tiling option_tiling(const Env& env, const std::vector<FilterJob>& jobs) {
  bool any_group = false, any_node = false;
  for (const auto& j : jobs) {
    any_group |= j.P->groups != nullptr;
    any_node |= j.P->nodes != nullptr;
  }
  const int rows = any_node && !any_group ? kRowsPerNodeBlock : kRowsPerBlock;
  return {env.opt.tile_rows > 0 ? env.opt.tile_rows : rows, env.opt.tile_wgs > 0 ? env.opt.tile_wgs : kWgPerXcd};
}

// Row-block fields of the Inst table and the grid for a tiling.  XCD x owns the
// row blocks [x * slab, (x + 1) * slab) of each pencil; the grid gives each XCD
// min(wgs, largest slab) workgroups.
void apply_tiling(std::vector<Inst>& insts, Batch& b, Tiling t) {
  int max_slab = 1;
  for (const Inst& I : insts) max_slab = std::max(max_slab, ((I.n + t.rpb - 1) / t.rpb + 7) / 8);
  const int per = std::max(1, std::min(t.wgs, max_slab));
  b.G = 8 * per;
  b.rows_per_block = t.rpb;
  for (Inst& I : insts) {
    I.nrb = (I.n + t.rpb - 1) / t.rpb;
    I.slab = (I.nrb + 7) / 8;
    I.steps = (I.slab + per - 1) / per;
    // spreads pencils smaller than the grid over the workgroups; depends on the
    // pencil and the grid only, so a pencil computes the same alone and in a batch
    I.rot = (int)((uint32_t)I.n * 2654435761u % (uint32_t)per);
  }
}

// Copies host bytes into `keep` (alive until the stream has passed the copy)
// and enqueues the upload.
hipError_t put_async(hipStream_t s, std::vector<std::vector<char>>& keep, void* dst, const void* src,
                     size_t bytes) {
  if (!bytes) return hipSuccess;
  keep.emplace_back((const char*)src, (const char*)src + bytes);
  return hipMemcpyAsync(dst, keep.back().data(), bytes, hipMemcpyHostToDevice, s);
}

// Builds and uploads the device tables of the batch: the Inst table (host copy
// left in `insts`), the tile and column owners, per-column and per-pole shifts,
// weights and the ILU(0) factors.  The host arrays are parked in `keep`, which
// the caller holds until the stream has passed the copies.
// Column order (col_pole): right-hand-side-major with warm starts (mixed
// precision, options.recycle), pole-major otherwise.
// Column order of the Krylov block: pole-major (0), so that the tiles of the
// poles whose solves converge first retire early.  The kernels also take the
// right-hand-side-major order (1), which paid with warm starts while every
// column had one inner target; with the columns beyond gamma solved loosely
// it is the slower one.
int column_order(const Env& env) {
  (void)env;
  return 0;
}

// Fills P.tables with the preconditioner factors of the pole set sigma (2N)
// in precision R, unless it already holds them: ILU(0) factors per pole, node
// block inverses per pole (block Jacobi and node SGS), the node SGS factors
// R and D per pole, or the point SGS factor R = sqrt(d) per (row, pole).
template <typename R>
slrf_status prec_tables(Env& env, const Pencil& P, int N, const double* sigma) {
  PrecTables& T = P.tables;
  const double om = sgs_omega_of(env, P);
  if (T.rsize == (int)sizeof(R) && T.omega == om && T.sigma.size() == (size_t)(2 * N) &&
      std::equal(T.sigma.begin(), T.sigma.end(), sigma))
    return SLRF_OK;
  T = PrecTables{};
  // Symmetric SOR: D / omega in place of the diagonal blocks D, so the sweeps
  // take (D / omega)^{-1} = omega D^{-1}, R with R R^T = D / omega, and
  // 2 D / omega - D = (2 / omega - 1) D where the split form subtracts D
  // (omega = 1: the plain SGS, every factor 1).
  const double s_inv = om, s_r = 1.0 / std::sqrt(om), s_d = 2.0 / om - 1.0;
  auto append = [](std::vector<char>& dst, const std::vector<std::complex<double>>& v) {
    const size_t o = dst.size();
    dst.resize(o + v.size() * sizeof(cx<R>));
    cx<R>* out = reinterpret_cast<cx<R>*>(dst.data() + o);
    for (size_t k = 0; k < v.size(); ++k) out[k] = {(R)v[k].real(), (R)v[k].imag()};
  };
  std::vector<std::complex<double>> f1, f2;
  for (int p = 0; p < N; ++p) {
    const std::complex<double> sg(sigma[2 * p], sigma[2 * p + 1]);
    if (P.use_ilu) {
      if (!ilu0_factor(P, sg, f1))
        return fail(env, SLRF_E_BREAKDOWN, "zero pivot in the ILU(0) factorisation of the shifted operator");
      f1.resize((size_t)P.nnz);
      append(T.ilu, f1);
    }
    if (P.use_bjac || P.sgs == 3) {
      if (!bjac3_factor(P, sg, f1)) return fail(env, SLRF_E_BREAKDOWN, "singular node block of the shifted operator");
      if (P.sgs == 3 && om != 1.0)
        for (auto& z : f1) z *= s_inv;
      append(T.bjac, f1);
    }
    if (P.sgs == 3) {
      if (!sgs3_factor(P, sg, f1, f2))
        return fail(env, SLRF_E_BREAKDOWN, "node block of the shifted operator without a symmetric factor");
      if (om != 1.0) {
        for (auto& z : f1) z *= s_r;
        for (auto& z : f2) z *= s_d;
      }
      append(T.sgsR, f1);
      append(T.sgsD, f2);
    }
  }
  if (P.sgs == 1) {
    // R = sqrt(d) per (row, pole), (n, N) layout; d itself is computed on the
    // device in the Krylov precision from the same diagonals
    std::vector<double> dA(P.n), dB(P.n);
    for (int64_t i = 0; i < P.n; ++i)
      for (int32_t q = P.h_rp[i]; q < P.h_rp[i + 1]; ++q)
        if (P.h_cl[q] == i) {
          dA[i] = P.h_ab[2 * (size_t)q];
          dB[i] = P.h_ab[2 * (size_t)q + 1];
        }
    f1.resize((size_t)P.n * N);
    for (int64_t i = 0; i < P.n; ++i)
      for (int p = 0; p < N; ++p)
        f1[(size_t)i * N + p] =
            std::sqrt(std::complex<double>(dA[i], 0.0) - std::complex<double>(sigma[2 * p], sigma[2 * p + 1]) * dB[i]);
    if (om != 1.0)
      for (auto& z : f1) z *= s_r;
    append(T.sgsR, f1);
  }
  T.rsize = (int)sizeof(R);
  T.omega = om;
  T.sigma.assign(sigma, sigma + 2 * N);
  return SLRF_OK;
}

// Each colour-sweep workgroup takes a share of a colour's nodes: the smallest
// multiple of 4 (the same count for each wavefront) that keeps the largest
// colour within a cap of workgroups.  A job with at least 8 column tiles (long
// launches, bound by bandwidth) takes the largest grid, 2048: more, smaller
// shares balance better than one resident generation (48^3 elasticity, 16
// tiles: 8 nodes per workgroup over 1728 workgroups, a full-width launch
// 1.63 ms against 1.77 ms for 13.5 over 1024).  Fewer tiles (short launches,
// bound by latency) stay within the 1024 resident workgroups (scalar pencils
// of n ~ 1e5 with 3 to 5 tiles: 4% faster than with the larger grid).  The
// share depends on the job alone, not on the batch.
void sgs_shares(const Pencil& P, int tiles, int& share, int& wgs) {
  share = 4;
  wgs = 0;
  if (!P.sgs || P.sgs_maxc < 1) return;  // no colour sweeps for this pencil
  const int64_t cap = tiles >= 8 ? kMaxGrid : 8 * kWgPerXcd;
  share = 4 * (int)((P.sgs_maxc + 4 * cap - 1) / (4 * cap));
  wgs = (int)((P.sgs_maxc + share - 1) / share);
}

template <typename R>
slrf_status upload_tables(Env& env, std::vector<FilterJob>& jobs, const FilterLayout& lo, Batch& b,
                          std::vector<Inst>& insts, std::vector<std::vector<char>>& keep) {
  const hipStream_t s = env.stream;
  insts.assign(jobs.size(), Inst{});
  b.V = lane_width(std::is_same<R, float>::value);
  // sparse-product variant: stencil groups if some pencil has them, else node
  // triples if some pencil has those (1 and 2, the kernels' row modes)
  bool any_group = false, any_node = false;
  for (const auto& j : jobs) {
    any_group |= j.P->groups != nullptr;
    any_node |= j.P->nodes != nullptr;
  }
  b.groups = any_group ? 1 : any_node ? 2 : 0;
  std::vector<int> tile_inst, col_inst;
  std::vector<cx<R>> sigc, sigj;
  struct Upload {
    char* dst;
    const char* src;  // a pencil's PrecTables, unchanged until the next application
    size_t bytes;
  };
  std::vector<Upload> uploads;
  std::vector<double> sigc64, w;
  int64_t dn = 0, ilu_off = 0, bjac_off = 0, sgs_off = 0, sgsd_off = 0;  // sgsd: node blocks' D only
  b.sgs = 0;
  b.sgs_ncol = 0;
  b.Gs = 8;
  int col0 = 0, tile0 = 0;
  for (size_t q = 0; q < jobs.size(); ++q) {
    const FilterJob& j = jobs[q];
    Inst& I = insts[q];
    I.n = (int)j.P->n;
    I.L = j.L;
    I.N = j.N;
    I.K = j.N * j.L;
    I.Kp = (int)padded_k(I.K, std::is_same<R, float>::value);
    I.col0 = col0;
    I.tile0 = tile0;
    I.nnz = (int)j.P->nnz;
    I.blk = j.blk;
    I.rl = j.rl;
    I.dn = dn;
    I.rowptr = j.P->rowptr;
    I.col = j.P->col;
    I.ab = std::is_same<R, float>::value ? (const void*)j.P->ab32 : (const void*)j.P->ab64;
    I.ab64 = j.P->ab64;
    I.sched = j.P->sched;
    I.groups = j.P->groups;
    I.nodes = j.P->nodes;
    I.diagpos = j.P->diagpos;
    I.ilu = nullptr;
    I.bjac = nullptr;
    I.sgs = j.P->sgs;
    I.sgs_ncol = j.P->sgs_ncol;
    sgs_shares(*j.P, I.Kp / (64 * b.V), I.sgs_share, I.sgs_wgs);
    I.sgs_cptr = j.P->sgs_cptr;
    I.sgs_nodes = j.P->sgs_nodes;
    I.lrp = j.P->lrp;
    I.lcol = j.P->lcol;
    I.urp = j.P->urp;
    I.ucol = j.P->ucol;
    I.lab = std::is_same<R, float>::value ? (const void*)j.P->lab32 : (const void*)j.P->lab64;
    I.uab = std::is_same<R, float>::value ? (const void*)j.P->uab32 : (const void*)j.P->uab64;
    I.sgsR = nullptr;
    I.sgsD = nullptr;
    const int tiles = (I.Kp + 64 * b.V - 1) / (64 * b.V);
    for (int t = 0; t < tiles; ++t) tile_inst.push_back((int)q);
    for (int c = 0; c < I.Kp; ++c) col_inst.push_back((int)q);
    for (int p = 0; p < j.N; ++p) {
      sigj.push_back({(R)j.sigma[2 * p], (R)j.sigma[2 * p + 1]});
      w.push_back(j.weight[2 * p]);
      w.push_back(j.weight[2 * p + 1]);
    }
    I.rmaj = column_order(env);
    for (int c = 0; c < I.K; ++c) {  // pole of column c in the pencil's column order
      const int p = col_pole(c, j.L, j.N, I.rmaj);
      sigc.push_back({(R)j.sigma[2 * p], (R)j.sigma[2 * p + 1]});
      sigc64.push_back(j.sigma[2 * p]);
      sigc64.push_back(j.sigma[2 * p + 1]);
    }
    for (int c = I.K; c < I.Kp; ++c) {  // padding columns take the last pole (never active)
      sigc.push_back(sigc.back());
      sigc64.push_back(sigc64[sigc64.size() - 2]);
      sigc64.push_back(sigc64[sigc64.size() - 2]);
    }
    slrf_status ts = prec_tables<R>(env, *j.P, j.N, j.sigma);
    if (ts != SLRF_OK) return ts;
    const PrecTables& T = j.P->tables;
    if (j.P->use_ilu) {
      I.ilu = (const char*)lo.ilu + ilu_off * sizeof(cx<R>);
      uploads.push_back({(char*)lo.ilu + ilu_off * sizeof(cx<R>), T.ilu.data(), T.ilu.size()});
      ilu_off += (int64_t)j.N * j.P->nnz;
    }
    if (j.P->use_bjac || j.P->sgs == 3) {
      I.bjac = (const char*)lo.bjac + bjac_off * sizeof(cx<R>);
      uploads.push_back({(char*)lo.bjac + bjac_off * sizeof(cx<R>), T.bjac.data(), T.bjac.size()});
      bjac_off += (int64_t)j.N * (j.P->n / 3) * 9;
    }
    if (j.P->sgs == 3) {
      I.sgsR = (const char*)lo.sgsR + sgs_off * sizeof(cx<R>);
      I.sgsD = (const char*)lo.sgsD + sgsd_off * sizeof(cx<R>);
      uploads.push_back({(char*)lo.sgsR + sgs_off * sizeof(cx<R>), T.sgsR.data(), T.sgsR.size()});
      uploads.push_back({(char*)lo.sgsD + sgsd_off * sizeof(cx<R>), T.sgsD.data(), T.sgsD.size()});
      sgs_off += (int64_t)j.N * (j.P->n / 3) * 9;
      sgsd_off += (int64_t)j.N * (j.P->n / 3) * 9;
    } else if (j.P->sgs == 1) {
      I.sgsR = (const char*)lo.sgsR + sgs_off * sizeof(cx<R>);
      uploads.push_back({(char*)lo.sgsR + sgs_off * sizeof(cx<R>), T.sgsR.data(), T.sgsR.size()});
      sgs_off += (int64_t)I.n * I.N;
    }
    if (j.P->sgs) {
      b.sgs |= j.P->sgs == 3 ? 2 : 1;
      b.sgs_ncol = std::max(b.sgs_ncol, j.P->sgs_ncol);
      b.Gs = std::max(b.Gs, (I.sgs_wgs + 7) / 8 * 8);
    }
    dn += (int64_t)I.n * I.N;
    col0 += I.Kp;
    tile0 += tiles;
  }
  b.inst = lo.inst;
  b.tile_inst = lo.tile_inst;
  b.col_inst = lo.col_inst;
  b.active = lo.active;
  b.n_active = lo.n_active;
  b.n_tiles = tile0;
  b.Ktot = col0;
  apply_tiling(insts, b, option_tiling(env, jobs));
  HIPCHK(env, put_async(s, keep, lo.inst, insts.data(), insts.size() * sizeof(Inst)));
  HIPCHK(env, put_async(s, keep, lo.tile_inst, tile_inst.data(), 4 * tile_inst.size()));
  HIPCHK(env, put_async(s, keep, lo.col_inst, col_inst.data(), 4 * col_inst.size()));
  HIPCHK(env, put_async(s, keep, lo.sigma_col, sigc.data(), sizeof(cx<R>) * sigc.size()));
  HIPCHK(env, put_async(s, keep, lo.sig_j, sigj.data(), sizeof(cx<R>) * sigj.size()));
  HIPCHK(env, put_async(s, keep, lo.w, w.data(), 8 * w.size()));
  if (lo.sigma_col64) HIPCHK(env, put_async(s, keep, lo.sigma_col64, sigc64.data(), 8 * sigc64.size()));
  for (const Upload& u : uploads)
    if (u.bytes) HIPCHK(env, hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, s));
  return SLRF_OK;
}

// ---------------------------------------------------------------------------
// Tile autotuner: for a batch shape not seen before in this process, times
// two BiCGStab iterations for each candidate tiling and keeps the fastest.
// The shape key is (precision, log2 of the column tiles, log2 of the rows,
// nonzeros per row to a factor sqrt(2)).

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, Tiling> g_tune_cache;

int ilog2(int64_t x) {
  int r = 0;
  while (x > 1) {
    x >>= 1;
    ++r;
  }
  return r;
}

// Inner-solver dispatch: start values after the right-hand side is in r, and one
// iteration (BiCGStab of the paper, or COCG with options.solver = 1).
template <typename R>
void krylov_start(const Env& env, const Batch& b, const KrylovState<R>& st) {
  if (env.opt.solver == 1)
    launch_cocg_start<R>(env.stream, b, st);
  else
    launch_init_scalars<R>(env.stream, b, st);
}

template <typename R>
void krylov_iteration(const Env& env, const Batch& b, const KrylovState<R>& st, R tol, int maxit, bool first,
                      int precs, LaunchTimer* tm, const IterBytes& by) {
  if (env.opt.solver == 1)
    launch_cocg_iteration<R>(env.stream, b, st, tol, maxit, first, tm, by);
  else
    launch_iteration<R>(env.stream, b, st, tol, maxit, first, precs, tm, by);
}

template <typename R>
slrf_status autotune(Env& env, std::vector<Inst>& insts, const FilterLayout& lo, Batch& b,
                     const KrylovState<R>& st, R tol, int precs, const IterBytes& by,
                     const std::function<void()>& restart, std::vector<std::vector<char>>& keep) {
  const hipStream_t s = env.stream;
  int64_t rows = 0, nnz = 0;
  for (const Inst& I : insts) {
    rows += I.n;
    nnz += I.nnz;
  }
  const auto key = std::make_tuple((int)sizeof(R), ilog2(b.n_tiles), ilog2(rows),
                                   (int)std::lround(2.0 * std::log2((double)nnz / (double)rows)));
  Tiling best{0, 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) best = it->second;
  }
  if (best.rpb == 0) {
    static const Tiling cands[] = {{16, 128}, {32, 128}, {8, 128}, {16, 256}, {32, 256}, {16, 64}, {24, 128},
                                   {48, 128}};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(env, hipEventCreate(&e0));
    HIPCHK(env, hipEventCreate(&e1));
    float best_ms = INFINITY;
    hipError_t err = hipSuccess;
    for (const Tiling& c : cands) {
      apply_tiling(insts, b, c);
      err = put_async(s, keep, lo.inst, insts.data(), insts.size() * sizeof(Inst));
      if (err != hipSuccess) break;
      restart();
      krylov_iteration<R>(env, b, st, tol, 1 << 30, true, precs, nullptr, by);
      (void)hipEventRecord(e0, s);
      for (int q = 0; q < 2; ++q) krylov_iteration<R>(env, b, st, tol, 1 << 30, false, precs, nullptr, by);
      (void)hipEventRecord(e1, s);
      err = hipEventSynchronize(e1);
      float ms = 0;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err != hipSuccess) break;
      if (env.verbose) fprintf(stderr, "[slrf] tune rows %d wgs %d: %.3f ms\n", c.rpb, c.wgs, ms);
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(env, SLRF_E_DEVICE, std::string("autotune: ") + hipGetErrorString(err));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  apply_tiling(insts, b, best);
  HIPCHK(env, put_async(s, keep, lo.inst, insts.data(), insts.size() * sizeof(Inst)));
  restart();
  HIPCHK(env, hipGetLastError());
  return SLRF_OK;
}

// Runs BiCGStab iterations on the batch until no column is active or maxit is
// reached, polling the active count every check_every iterations.  With
// opt.graph (no profiling, a non-null stream) one chunk of check_every
// iterations plus the count is captured once as a hipGraph and replayed.
template <typename R>
slrf_status run_krylov(Env& env, const Batch& b, const KrylovState<R>& st, R tol, int precs, const IterBytes& by,
                       int* d_count, slrf_filter_stats* ks) {
  const hipStream_t s = env.stream;
  const int maxit = std::max(1, env.opt.inner_maxit);
  const int every = std::max(1, std::min(env.opt.check_every, 64));
  LaunchTimer* tm = env.opt.profile ? &env.timer : nullptr;
  const bool graph = env.opt.graph && !tm && s != nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t gr = nullptr;
  slrf_status out = SLRF_OK;
  int it = 0;
  auto cleanup = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (gr) (void)hipGraphDestroy(gr);
  };
  while (it < maxit) {
    const int chunk = std::min(every, maxit - it);
    if (graph && it > 0 && chunk == every) {
      if (!exec) {
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          for (int q = 0; q < every; ++q) krylov_iteration<R>(env, b, st, tol, maxit, false, precs, nullptr, by);
          launch_count_active(s, b, st.flags, d_count);
          e = hipStreamEndCapture(s, &gr);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) {
          cleanup();
          return fail(env, SLRF_E_DEVICE, std::string("hipGraph capture: ") + hipGetErrorString(e));
        }
      }
      hipError_t e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) {
        cleanup();
        return fail(env, SLRF_E_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
      }
      it += every;
    } else {
      for (int q = 0; q < chunk; ++q, ++it) krylov_iteration<R>(env, b, st, tol, maxit, it == 0, precs, tm, by);
      launch_count_active(s, b, st.flags, d_count);
    }
    int active = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&active, d_count, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      cleanup();
      return fail(env, SLRF_E_DEVICE, std::string("Krylov iteration: ") + hipGetErrorString(e));
    }
    if (tm) {
      out = harvest_timer(env, b.G, (int64_t)b.n_tiles, (int64_t)b.Ktot, ks);
      if (out != SLRF_OK) break;
    }
    if (active == 0) break;
  }
  cleanup();
  return out;
}

IterBytes iter_bytes(const std::vector<FilterJob>& jobs, const FilterLayout& lo, size_t rs, bool complex_rhat) {
  IterBytes by{};
  for (const auto& j : jobs) by.blk += (double)j.P->n * j.N * j.L * 2 * rs;  // padding excluded
  by.rhat = complex_rhat ? by.blk : (double)lo.ER * rs;
  by.diag = (double)lo.ED * 2 * rs;
  for (const auto& j : jobs) by.matrix += merged_csr_bytes(*j.P, 2 * rs);
  for (const auto& j : jobs)
    if (j.P->sgs) {
      // column index plus (a, b) pair per coupling, and the row pointers
      by.sgs_lower += (double)j.P->lnnz * (4 + 2 * rs) + 4.0 * (j.P->n + 1);
      by.sgs_upper += (double)j.P->unnz * (4 + 2 * rs) + 4.0 * (j.P->n + 1);
      // R, D and D^{-1} for every pole (point: D and D^{-1} are the diagonal blocks)
      by.sgs_blocks += (double)j.N * j.P->n * (j.P->sgs == 3 ? 3.0 * 3 : 3.0) * 2 * rs;
    }
  return by;
}

// Per-column outcome of a finished BiCGStab run, summed per job.  sum_it gets
// each job's total iteration count; with final_relres the recursive residual
// ratio rnorm / fnorm feeds max_relres.
template <typename R>
slrf_status collect_stats(Env& env, std::vector<FilterJob>& jobs, const KrylovState<R>& st, int64_t Ktot,
                          bool final_relres, std::vector<double>& sum_it) {
  std::vector<int> fl(Ktot), its(Ktot);
  std::vector<R> rn(Ktot), fn(Ktot);
  HIPCHK(env, hipMemcpyAsync(fl.data(), st.flags, 4 * (size_t)Ktot, hipMemcpyDeviceToHost, env.stream));
  HIPCHK(env, hipMemcpyAsync(its.data(), st.iters, 4 * (size_t)Ktot, hipMemcpyDeviceToHost, env.stream));
  HIPCHK(env, hipMemcpyAsync(rn.data(), st.rnorm, sizeof(R) * (size_t)Ktot, hipMemcpyDeviceToHost, env.stream));
  HIPCHK(env, hipMemcpyAsync(fn.data(), st.fnorm, sizeof(R) * (size_t)Ktot, hipMemcpyDeviceToHost, env.stream));
  HIPCHK(env, hipStreamSynchronize(env.stream));
  sum_it.assign(jobs.size(), 0.0);
  int64_t c = 0;
  for (size_t q = 0; q < jobs.size(); ++q) {
    slrf_filter_stats& fs = jobs[q].stats;
    const int K = jobs[q].N * jobs[q].L;
    const int Kp = (int)padded_k(K, sizeof(R) == 4);
    for (int k = 0; k < Kp; ++k, ++c) {
      if (k >= K) continue;
      fs.max_iterations = std::max(fs.max_iterations, its[c]);
      sum_it[q] += its[c];
      // BiCGStab: two products per iteration (one at a half-step exit); COCG: one
      fs.spmv += env.opt.solver == 1 ? (int64_t)its[c] : 2 * (int64_t)its[c] - (fl[c] == COL_HALF_CONVERGED ? 1 : 0);
      if (fl[c] == COL_BREAKDOWN) fs.n_breakdown++;
      if (fl[c] == COL_MAXIT) fs.n_maxit++;
      if (final_relres) fs.max_relres = std::max(fs.max_relres, fn[c] > 0 ? (double)rn[c] / (double)fn[c] : 0.0);
    }
  }
  return SLRF_OK;
}

// job_rounds (mixed precision): the correction rounds in which each job had
// an open column
void finish_stats(std::vector<FilterJob>& jobs, const std::vector<double>& sum_it, const slrf_filter_stats& ks,
                  double seconds, const std::vector<int>* job_rounds) {
  for (size_t q = 0; q < jobs.size(); ++q) {
    slrf_filter_stats& fs = jobs[q].stats;
    fs.mean_iterations = sum_it[q] / std::max(1, jobs[q].N * jobs[q].L);
    fs.refinements = job_rounds ? (*job_rounds)[q] : 0;
    fs.seconds = seconds;
    fs.spmm_seconds = ks.spmm_seconds;
    fs.spmm_launches = ks.spmm_launches;
    fs.spmm_bytes = ks.spmm_bytes;
    fs.spmm_columns = ks.spmm_columns;
    fs.update_seconds = ks.update_seconds;
    fs.update_launches = ks.update_launches;
    fs.update_bytes = ks.update_bytes;
  }
}

// FP64 filter application: every (job, pole, column) system solved by
// BiCGStab in complex FP64 with x0 = 0 and shadow residual B X, then
// U = sum_j 2 Re(w_j Y_j) per job.
slrf_status filter_batch_fp64(Env& env, Carver& arena, std::vector<FilterJob>& jobs) {
  const double t0 = now_s();
  const hipStream_t s = env.stream;
  std::vector<JobShape> js;
  for (auto& j : jobs) js.push_back({j.P->n, j.P->nnz, j.L, j.N, j.P->use_ilu, false, j.P->use_bjac, j.P->sgs});
  FilterLayout lo;
  carve_filter(arena, js, false, lo);
  place_jobs(jobs, false);
  if (arena.off > arena.cap) return fail(env, SLRF_E_WORKSPACE, "workspace too small for this L and pole count");
  Batch b{};
  std::vector<std::vector<char>> keep;
  std::vector<Inst> insts;
  slrf_status st0 = upload_tables<double>(env, jobs, lo, b, insts, keep);
  if (st0 != SLRF_OK) return st0;
  KrylovState<double> st = make_state<double>(lo);
  int64_t dn = 0, pj = 0;
  for (auto& j : jobs) {
    launch_jacobi_diag<double>(s, (int)j.P->n, j.N, j.P->diagA, j.P->diagB, (const cx<double>*)lo.sig_j + pj,
                               (cx<double>*)lo.d + dn, (cx<double>*)lo.dinv + dn, point_sgs_cd(env, *j.P),
                               point_sgs_ci(env, *j.P));
    launch_spmm_real<double>(s, (int)j.P->n, j.L, j.P->rowptr, j.P->col, j.P->ab64, j.X, nullptr, lo.rhat + j.rl);
    dn += j.P->n * j.N;
    pj += j.N;
  }
  launch_init<double>(s, b, st, lo.rhat);
  krylov_start<double>(env, b, st);
  HIPCHK(env, hipGetLastError());
  slrf_filter_stats ks{};
  const IterBytes by = iter_bytes(jobs, lo, 8, false);
  if (env.opt.tune) {
    slrf_status ts = autotune<double>(env, insts, lo, b, st, env.opt.inner_tol, lo.precs(), by, [&]() {
      launch_init<double>(s, b, st, lo.rhat);
      krylov_start<double>(env, b, st);
    }, keep);
    if (ts != SLRF_OK) return ts;
  }
  slrf_status rs = run_krylov<double>(env, b, st, env.opt.inner_tol, lo.precs(), by, lo.count, &ks);
  if (rs != SLRF_OK) return rs;
  if (b.sgs) launch_sgs_finish<double>(s, b, st);  // x = M_L^{-T} x' for every column
  int64_t wj = 0;
  for (auto& j : jobs) {
    launch_filter_sum<double>(s, (int)j.P->n, j.L, j.N, tile_width(false), column_order(env), st.x + j.blk,
                              lo.w + 2 * wj, j.U, false);
    wj += j.N;
  }
  HIPCHK(env, hipGetLastError());
  for (auto& j : jobs) j.stats = slrf_filter_stats{};
  std::vector<double> sum_it;
  slrf_status cs = collect_stats<double>(env, jobs, st, lo.Ktot, true, sum_it);
  if (cs != SLRF_OK) return cs;
  finish_stats(jobs, sum_it, ks, now_s() - t0, nullptr);
  return SLRF_OK;
}

// Filter application with complex FP32 inner solves and FP64 defect correction:
//   Y = 0; repeat { R = F - S Y in FP64; stop the columns with
//   ||R|| <= target ||F||; solve S D = R / ||R|| in FP32 by BiCGStab to relative
//   residual clamp(0.1 target ||F|| / ||R||, 1e-6, 1e-1); Y += ||R|| D };
//   U = sum_j 2 Re(w_j Y_j).
// Warm starts (jobs with warm set): Y starts from Y_prev C instead of 0, and
// the rounds start from the defect of that start; in such an application the
// other jobs start from Y = 0 through the same steps, which computes what
// their cold start computes.  Jobs with yprev keep Y and B X for the next one.
slrf_status filter_batch_mixed(Env& env, Carver& arena, std::vector<FilterJob>& jobs) {
  const double t0 = now_s();
  const hipStream_t s = env.stream;
  std::vector<JobShape> js;
  for (auto& j : jobs) js.push_back({j.P->n, j.P->nnz, j.L, j.N, j.P->use_ilu, false, j.P->use_bjac, j.P->sgs});
  FilterLayout lo;
  carve_filter(arena, js, true, lo);
  place_jobs(jobs, true);
  if (arena.off > arena.cap) return fail(env, SLRF_E_WORKSPACE, "workspace too small for this L and pole count");
  Batch b{};
  std::vector<std::vector<char>> keep;
  std::vector<Inst> insts;
  slrf_status st0 = upload_tables<float>(env, jobs, lo, b, insts, keep);
  if (st0 != SLRF_OK) return st0;
  KrylovState<float> st = make_state<float>(lo);
  // Per column: the FP64 defect target of its job.  The relative tolerance of
  // each FP32 correction solve is set per column by the defect kernel from the
  // gap between the current defect and that target.
  std::vector<double> tol_host;
  for (auto& j : jobs)
    for (int64_t c = 0; c < padded_k(j.N * j.L, true); ++c)
      tol_host.push_back(j.rhs_target && c < j.N * j.L ? j.rhs_target[col_rhs((int)c, j.L, j.N, column_order(env))]
                                                       : j.target);
  const float tol32 = (float)kInnerTol32;  // unused: every column has its own
  HIPCHK(env, put_async(s, keep, lo.tol64, tol_host.data(), 8 * tol_host.size()));
  st.tolc = lo.tol32;
  bool warm = false;
  for (const auto& j : jobs) warm = warm || j.warm;
  if (warm) {
    // Y0 = Y_prev C with C = X_prev^T B X_new = F_prev^T X_new (Y0 = 0 for the
    // jobs without a previous application)
    for (auto& j : jobs) {
      const int n = (int)j.P->n;
      const int64_t Kp = padded_k(j.N * j.L, true);
      if (j.warm) {
        launch_gram(s, n, j.L, j.fprev, j.X, j.X, j.gpart, j.nch, j.C, j.Cb);
        launch_recycle(s, n, j.L, j.N, tile_width(true), (int)Kp, column_order(env), j.yprev, j.C, lo.Y + j.blk);
      } else {
        launch_fill_zero(s, lo.Y + j.blk, (size_t)n * Kp * sizeof(cx<double>));
      }
    }
    HIPCHK(env, hipGetLastError());
  }
  int64_t dn = 0, pj = 0;
  for (auto& j : jobs) {
    launch_jacobi_diag<float>(s, (int)j.P->n, j.N, j.P->diagA32, j.P->diagB32, (const cx<float>*)lo.sig_j + pj,
                              (cx<float>*)lo.d + dn, (cx<float>*)lo.dinv + dn, point_sgs_cd(env, *j.P),
                              point_sgs_ci(env, *j.P));
    launch_spmm_real<double>(s, (int)j.P->n, j.L, j.P->rowptr, j.P->col, j.P->ab64, j.X, nullptr, lo.F + j.rl);
    dn += j.P->n * j.N;
    pj += j.N;
  }
  HIPCHK(env, hipGetLastError());
  const IterBytes by = iter_bytes(jobs, lo, 4, true);
  slrf_filter_stats ks{};
  for (auto& j : jobs) j.stats = slrf_filter_stats{};
  std::vector<double> sum_it(jobs.size(), 0.0), it_round;
  int rounds = 0;
  if (warm) {
    // ||F|| of every column (the targets are relative to it); the rounds then
    // start from the defect of the warm start
    launch_defect(s, b, lo.sigma_col64, lo.F, nullptr, lo.R, lo.part64, lo.scale);
    launch_defect_norms(s, b, lo.part64, lo.tol64, 1, lo.fnorm64, lo.scale, lo.relres, lo.tol32, kInnerTol32,
                        lo.count);
  }
  // rounds round0 .. last: up to kMaxRounds correction solves, then the defect
  // of the last one
  const int round0 = warm ? 1 : 0, last = kMaxRounds + round0;
  // per job: an open column entering the round (the defect then computes its
  // product with S; the counts match the job's solve alone)
  std::vector<char> job_open(jobs.size(), 1);
  std::vector<int> job_rounds(jobs.size(), 0);
  std::vector<double> scale_h(lo.Ktot);
  for (int round = round0; round <= last; ++round) {
    launch_defect(s, b, lo.sigma_col64, lo.F, round ? lo.Y : nullptr, lo.R, lo.part64, lo.scale);
    launch_defect_norms(s, b, lo.part64, lo.tol64, round == 0, lo.fnorm64, lo.scale, lo.relres, lo.tol32,
                        kInnerTol32, lo.count);
    HIPCHK(env, hipGetLastError());
    int open = 0;
    HIPCHK(env, hipMemcpyAsync(&open, lo.count, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(env, hipMemcpyAsync(scale_h.data(), lo.scale, 8 * (size_t)lo.Ktot, hipMemcpyDeviceToHost, s));
    HIPCHK(env, hipStreamSynchronize(s));
    int64_t c0 = 0;
    for (size_t q = 0; q < jobs.size(); ++q) {
      const int K = jobs[q].N * jobs[q].L;
      // the defect's product with S (not counted for a zero start, which a cold
      // start does not compute)
      if (round > 0 && job_open[q] && (jobs[q].warm || round > round0)) jobs[q].stats.spmv += K;
      bool any = false;
      for (int k = 0; k < K && !any; ++k) any = scale_h[c0 + k] > 0;
      job_open[q] = any;
      c0 += padded_k(K, true);
    }
    if (open == 0 || round == last) break;
    ++rounds;
    for (size_t q = 0; q < jobs.size(); ++q) job_rounds[q] += job_open[q];
    launch_mixed_rhs(s, b, round ? lo.R : nullptr, lo.F, lo.scale, st, (cx<float>*)lo.vec[8]);
    krylov_start<float>(env, b, st);
    if (round == round0 && env.opt.tune) {
      slrf_status ts = autotune<float>(env, insts, lo, b, st, tol32, lo.precs(), by, [&]() {
        launch_mixed_rhs(s, b, round ? lo.R : nullptr, lo.F, lo.scale, st, (cx<float>*)lo.vec[8]);
        krylov_start<float>(env, b, st);
      }, keep);
      if (ts != SLRF_OK) return ts;
    }
    slrf_status rs = run_krylov<float>(env, b, st, tol32, lo.precs(), by, lo.count, &ks);
    if (rs != SLRF_OK) return rs;
    if (b.sgs) launch_sgs_finish<float>(s, b, st);  // x = M_L^{-T} x' for every column
    launch_accumulate(s, b, st.x, lo.scale, lo.Y, round == 0);
    slrf_status cs = collect_stats<float>(env, jobs, st, lo.Ktot, false, it_round);
    if (cs != SLRF_OK) return cs;
    for (size_t q = 0; q < jobs.size(); ++q) sum_it[q] += it_round[q];
  }
  int64_t wj = 0;
  for (auto& j : jobs) {
    const int64_t Kp = padded_k(j.N * j.L, true);
    if (rounds > 0 || warm) {
      launch_filter_sum<double>(s, (int)j.P->n, j.L, j.N, tile_width(true), column_order(env), lo.Y + j.blk,
                                lo.w + 2 * wj, j.U, false);
    } else {  // every column met its target with Y = 0
      HIPCHK(env, hipMemsetAsync(j.U, 0, 8 * (size_t)j.P->n * j.L, s));
      launch_fill_zero(s, lo.Y + j.blk, (size_t)j.P->n * Kp * sizeof(cx<double>));
    }
    if (j.yprev) {
      HIPCHK(env, hipMemcpyAsync(j.yprev, lo.Y + j.blk, (size_t)j.P->n * Kp * sizeof(cx<double>),
                                 hipMemcpyDeviceToDevice, s));
      HIPCHK(env, hipMemcpyAsync(j.fprev, lo.F + j.rl, (size_t)j.P->n * j.L * 8, hipMemcpyDeviceToDevice, s));
    }
    wj += j.N;
  }
  HIPCHK(env, hipGetLastError());
  std::vector<double> rr(lo.Ktot);
  HIPCHK(env, hipMemcpyAsync(rr.data(), lo.relres, 8 * (size_t)lo.Ktot, hipMemcpyDeviceToHost, s));
  HIPCHK(env, hipStreamSynchronize(s));
  int64_t c = 0;
  for (size_t q = 0; q < jobs.size(); ++q) {
    const int K = jobs[q].N * jobs[q].L;
    for (int k = 0; k < padded_k(K, true); ++k, ++c)
      if (k < K) jobs[q].stats.max_relres = std::max(jobs[q].stats.max_relres, rr[c]);
  }
  finish_stats(jobs, sum_it, ks, now_s() - t0, &job_rounds);
  return SLRF_OK;
}

slrf_status filter_batch(Env& env, Carver& arena, std::vector<FilterJob>& jobs) {
  if (jobs.empty()) return SLRF_OK;
  return env.opt.precision == SLRF_MIXED ? filter_batch_mixed(env, arena, jobs) : filter_batch_fp64(env, arena, jobs);
}

// ---------------------------------------------------------------------------
// Outer iteration (Algorithm 1) per pencil

// Per-pencil device buffers of the outer iteration; warm (mixed precision with
// warm starts): also the previous filter application's Y (complex FP64, the
// mixed form's tile-major layout for up to N poles) and B X.
size_t outer_bytes(int64_t n, int64_t L, int64_t N, bool warm) {
  const int nch = gram_chunks((int)n, (int)L);
  const int64_t nrr = (n + 255) / 256;
  size_t b = 0;
  b += 5 * al((size_t)n * L * 8);              // V U WA WB X
  b += al((size_t)nch * 2 * L * L * 8);        // Gram partials
  b += 3 * al((size_t)L * L * 8);              // GA GB Z
  b += al((size_t)L * 8);                      // theta
  b += al((size_t)(nrr * 2 * L + 2 * L) * 8);  // residual partials
  if (warm) b += al((size_t)n * padded_k(N * L, true) * 16) + al((size_t)n * L * 8);  // Y_prev, B X_prev
  return b;
}

struct SolveJob {
  Pencil* P = nullptr;
  int L = 0, N = 0;
  double gamma = 0;
  std::vector<double> sig, w;  // host, 2N each
  char* mem = nullptr;         // mem_bytes = outer_bytes(n, L, N, warm) of device buffers
  size_t mem_bytes = 0;
  double *V = nullptr, *U = nullptr, *WA = nullptr, *WB = nullptr, *X = nullptr, *part = nullptr, *GA = nullptr,
         *GB = nullptr, *Zd = nullptr, *th = nullptr, *rpart = nullptr;
  cx<double>* Yprev = nullptr;  // warm starts: Y of the previous filter application
  double* Fprev = nullptr;      // and its right-hand side B X
  std::vector<double> rhs_tgt;  // per right-hand side inner accuracy of the next application
  bool has_prev = false;        // Yprev and Fprev hold the previous outer iteration's
  int nch = 0, nrr = 0;
  int k = 0, prev_count = -1, count = 0;
  double prev_maxr = INFINITY, prev_prev = INFINITY, mix_c = 3e-3, iter_sum = 0, t0 = 0;
  bool done = false;
  slrf_status status = SLRF_OK;
  std::string msg;
  std::vector<double> theta, rho;
  slrf_solve_stats ss{};

  // max_N: the pole count the buffers are sized for; warm: keep Yprev, Fprev
  void carve(char* m, int max_N, bool warm) {
    mem = m;
    const int64_t n = P->n;
    nch = gram_chunks((int)n, L);
    nrr = (int)((n + 255) / 256);
    mem_bytes = outer_bytes(n, L, max_N, warm);
    Carver co{m, 0, mem_bytes};
    V = co.take<double>((size_t)n * L);
    U = co.take<double>((size_t)n * L);
    WA = co.take<double>((size_t)n * L);
    WB = co.take<double>((size_t)n * L);
    X = co.take<double>((size_t)n * L);
    part = co.take<double>((size_t)nch * 2 * L * L);
    GA = co.take<double>((size_t)L * L);
    GB = co.take<double>((size_t)L * L);
    Zd = co.take<double>((size_t)L * L);
    th = co.take<double>(L);
    rpart = co.take<double>((size_t)nrr * 2 * L + 2 * L);
    if (warm) {
      Yprev = co.take<cx<double>>((size_t)n * padded_k((int64_t)max_N * L, true));
      Fprev = co.take<double>((size_t)n * L);
    }
  }
};

// Runs f(q) for q < count on up to the host's hardware threads (the L x L
// projected eigenproblems of the pencils of a step are independent).
void parallel_for(int count, const std::function<void(int)>& f) {
  const int nt = std::min<int>(count, std::max(1u, std::thread::hardware_concurrency()));
  if (nt <= 1) {
    for (int q = 0; q < count; ++q) f(q);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&]() {
      for (int q = next++; q < count; q = next++) f(q);
    });
  for (auto& th : pool) th.join();
}

// One Rayleigh-Ritz pass for every pencil of a step (Section 3,
// B-orthonormalisation by the projected pencil): Y = Xin Z with
// Z^T (Xin^T A Xin) Z = diag(theta), Z^T (Xin^T B Xin) Z = I.  The products and
// Gram kernels of all pencils are queued, then one synchronisation, then the
// projected eigenproblems run in parallel host threads, then the updates.
// f32[q]: pencil q's two Gram products on FP32 MFMA (FP32 inputs, FP32
// accumulation), for the first projection of a mixed-precision outer iteration
// whose Ritz pairs are still far from converged.  The update Y = Xin Z stays
// FP64 whatever Z is, so span(Y) = span(Xin) to FP64 rounding and the FP64 pass
// that follows sees the filtered subspace itself; only how nearly B-orthonormal
// Y comes out depends on the FP32 Gram.
// Host Z buffers are kept in zs until the caller's next synchronisation.
slrf_status rr_pass_all(Env& env, const std::vector<SolveJob*>& js, const std::vector<const double*>& Xin,
                        const std::vector<double*>& Y, const std::vector<char>& f32,
                        std::vector<std::vector<double>>& thetas, std::vector<std::vector<double>>& zs) {
  const hipStream_t s = env.stream;
  const int m = (int)js.size();
  std::vector<std::vector<double>> hA(m), hB(m);
  for (int q = 0; q < m; ++q) {
    SolveJob& J = *js[q];
    const int n = (int)J.P->n, L = J.L;
    launch_spmm_real<double>(s, n, L, J.P->rowptr, J.P->col, J.P->ab64, Xin[q], J.WA, J.WB);
    launch_gram(s, n, L, Xin[q], J.WA, J.WB, J.part, J.nch, J.GA, J.GB, f32[q] != 0);
    hA[q].resize((size_t)L * L);
    hB[q].resize((size_t)L * L);
    HIPCHK(env, hipMemcpyAsync(hA[q].data(), J.GA, 8 * hA[q].size(), hipMemcpyDeviceToHost, s));
    HIPCHK(env, hipMemcpyAsync(hB[q].data(), J.GB, 8 * hB[q].size(), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(env, hipGetLastError());
  HIPCHK(env, hipStreamSynchronize(s));
  thetas.assign(m, {});
  zs.assign(m, {});
  std::vector<char> ok(m, 0);
  parallel_for(m, [&](int q) {
    const int L = js[q]->L;
    thetas[q].assign(L, 0.0);
    zs[q].assign((size_t)L * L, 0.0);
    ok[q] = projected_pencil(L, hA[q].data(), hB[q].data(), thetas[q].data(), zs[q].data(),
                             f32[q] ? kF32GramFloor : 1e-15);
  });
  for (int q = 0; q < m; ++q)
    if (!ok[q]) return fail(env, SLRF_E_BREAKDOWN, "projected pencil not solvable (non-finite or zero Gram matrix)");
  for (int q = 0; q < m; ++q) {
    SolveJob& J = *js[q];
    HIPCHK(env, hipMemcpyAsync(J.Zd, zs[q].data(), 8 * zs[q].size(), hipMemcpyHostToDevice, s));
    const double* xs[1] = {Xin[q]};
    double* ys[1] = {Y[q]};
    launch_gemm_nz(s, (int)J.P->n, J.L, J.L, 1, xs, J.Zd, ys);
  }
  HIPCHK(env, hipGetLastError());
  return SLRF_OK;
}

// Rayleigh-Ritz (two passes), residuals rho_i and the stopping test of one
// outer iteration for the pencils of a step, after the filter has written
// their U.
slrf_status finish_outer_all(Env& env, const std::vector<SolveJob*>& js, const std::vector<FilterJob>& fj) {
  const hipStream_t s = env.stream;
  const int m = (int)js.size();
  for (int q = 0; q < m; ++q) {
    SolveJob& J = *js[q];
    const slrf_filter_stats& fs = fj[q].stats;
    J.ss.filter_seconds += fs.seconds;
    J.ss.spmv_total += fs.spmv;
    J.iter_sum += fs.mean_iterations;
    slrf_filter_stats& kk = J.ss.kernels;
    kk.spmm_seconds += fs.spmm_seconds;
    kk.spmm_launches += fs.spmm_launches;
    kk.spmm_bytes += fs.spmm_bytes;
    kk.spmm_columns += fs.spmm_columns;
    kk.update_seconds += fs.update_seconds;
    kk.update_launches += fs.update_launches;
    kk.update_bytes += fs.update_bytes;
  }
  // Two projections.  In mixed precision the first one forms its Gram
  // matrices on FP32 MFMA while the previous residuals exceed 1e-6 (before the
  // first outer iteration they count as infinite): it only has to
  // B-orthonormalise approximately.  The second, which gives the Ritz pairs,
  // the residuals and the count, is always FP64.
  std::vector<const double*> x1(m), x2(m);
  std::vector<double*> y1(m), y2(m);
  std::vector<char> f32(m, 0), f64(m, 0);
  for (int q = 0; q < m; ++q) {
    SolveJob& J = *js[q];
    x1[q] = J.U;
    y1[q] = J.X;
    x2[q] = J.X;
    y2[q] = J.V;
    f32[q] = env.opt.precision == SLRF_MIXED && J.prev_maxr > kFirstPassF32Above;
  }
  std::vector<std::vector<double>> th1, z1, th2, z2;
  slrf_status st = rr_pass_all(env, js, x1, y1, f32, th1, z1);
  if (st != SLRF_OK) return st;
  st = rr_pass_all(env, js, x2, y2, f64, th2, z2);
  if (st != SLRF_OK) return st;
  std::vector<std::vector<double>> sums(m);
  for (int q = 0; q < m; ++q) {
    SolveJob& J = *js[q];
    const int n = (int)J.P->n, L = J.L;
    J.theta = th2[q];
    launch_spmm_real<double>(s, n, L, J.P->rowptr, J.P->col, J.P->ab64, J.V, J.WA, J.WB);
    HIPCHK(env, hipMemcpyAsync(J.th, J.theta.data(), 8 * (size_t)L, hipMemcpyHostToDevice, s));
    launch_resid(s, n, L, J.WA, J.WB, J.th, J.rpart, J.nrr);
    sums[q].resize(2 * L);
    HIPCHK(env, hipMemcpyAsync(sums[q].data(), J.rpart + (size_t)J.nrr * 2 * L, 16 * (size_t)L,
                               hipMemcpyDeviceToHost, s));
  }
  HIPCHK(env, hipGetLastError());
  HIPCHK(env, hipStreamSynchronize(s));  // also the lifetime of the host Z buffers
  for (int q = 0; q < m; ++q) {
    SolveJob& J = *js[q];
    const int n = (int)J.P->n, L = J.L;
    J.rho.assign(L, 0.0);
    int count = 0;
    bool all_ok = true;
    double maxr = 0;
    for (int c = 0; c < L; ++c) {
      J.rho[c] = std::sqrt(sums[q][c]) / (std::fabs(J.theta[c]) * std::sqrt(sums[q][L + c]));
      if (J.theta[c] > 0 && J.theta[c] <= J.gamma) {
        ++count;
        maxr = std::max(maxr, J.rho[c]);
        if (!(J.rho[c] <= env.opt.outer_tol)) all_ok = false;
      }
    }
    J.count = count;
    J.ss.max_resid = maxr;
    J.prev_prev = J.prev_maxr;
    J.prev_maxr = count ? maxr : INFINITY;
    const slrf_filter_stats& fs = fj[q].stats;
    if (env.verbose)
      fprintf(stderr,
              "[slrf] n=%d outer %d: inner its mean %.1f max %d (rounds %d, maxit %d, breakdown %d, max relres "
              "%.2e) theta [%.6g, %.6g] count %d max rho %.3e\n",
              n, J.k, fs.mean_iterations, fs.max_iterations, fs.refinements, fs.n_maxit, fs.n_breakdown,
              fs.max_relres, J.theta[0], J.theta[L - 1], count, maxr);
    if (count == L) {
      J.done = true;
      J.status = SLRF_E_SUBSPACE_TOO_SMALL;
      J.msg = "all L Ritz values lie in (0, gamma]: increase L";
    } else if (count == J.prev_count && all_ok) {
      J.done = true;
      J.status = SLRF_OK;
    } else if (J.k >= std::max(1, env.opt.outer_maxit)) {
      J.done = true;
      J.status = SLRF_E_NOT_CONVERGED;
      J.msg = "outer iteration limit reached";
    }
    J.prev_count = count;
    if (J.done) {
      J.ss.outer_iterations = J.k;
      J.ss.inner_iterations = J.iter_sum / std::max(1, J.k);
      int found = 0;
      for (int c = 0; c < L; ++c)
        if (J.theta[c] > 0 && J.theta[c] <= J.gamma && J.rho[c] <= env.opt.outer_tol) ++found;
      J.ss.n_found = found;
      J.ss.seconds = now_s() - J.t0;
    }
  }
  return SLRF_OK;
}

// One outer step for every job not yet done: one batched filter application
// over all of them, then Rayleigh-Ritz and residuals per job.  A failure marks
// the jobs of the step done with that status.
// Warm starts across outer steps (options.recycle, mixed precision): each
// pencil keeps its last filter application's Y and B X in its own buffers, so
// it warm-starts from them in any later step, whichever pencils share the step.
slrf_status outer_step(Env& env, Carver arena, const std::vector<SolveJob*>& jobs) {
  std::vector<FilterJob> fj;
  std::vector<SolveJob*> act;
  for (SolveJob* J : jobs) {
    if (J->done) continue;
    ++J->k;
    double target = env.opt.inner_tol;
    if (env.opt.precision == SLRF_MIXED) {
      // Inner accuracy follows the outer residual: target = c * (largest
      // residual of the previous outer iteration), within [1e-13, 1e-3]
      // (c = 3e-3 at first).  The residual of a Ritz pair amplifies the inner
      // error by up to about lambda_max / theta, so when an outer iteration
      // fails to cut the residual 3x, c shrinks 100x.
      if (J->prev_prev < INFINITY && J->prev_maxr > 0.3 * J->prev_prev) J->mix_c = std::max(1e-9, J->mix_c * 1e-2);
      target = std::max(1e-13, std::min(1e-3, J->mix_c * J->prev_maxr));
    }
    fj.push_back({J->P, J->L, J->N, J->sig.data(), J->w.data(), J->V, J->U, target, nullptr, {}, J->part, J->GA,
                  J->GB, J->nch});
    FilterJob& f = fj.back();
    if (env.opt.precision == SLRF_MIXED && (int)J->theta.size() == J->L) {
      // The columns of V are the Ritz vectors of the previous step, by value.
      // Those beyond gamma only widen the subspace, and an inexact solve for
      // them leaves the wanted directions in its span: they are solved to
      // kBeyondGammaTarget (or the step's target if that is looser).
      J->rhs_tgt.assign(J->L, target);
      for (int l = 0; l < J->L; ++l)
        if (J->theta[l] > J->gamma) J->rhs_tgt[l] = std::max(target, kBeyondGammaTarget);
      f.rhs_target = J->rhs_tgt.data();
    }
    if (env.opt.recycle && env.opt.precision == SLRF_MIXED && J->Yprev) {
      f.yprev = J->Yprev;
      f.fprev = J->Fprev;
      f.warm = J->has_prev;
    }
    act.push_back(J);
  }
  if (act.empty()) return SLRF_OK;
  slrf_status st = filter_batch(env, arena, fj);
  // Y_prev (X_prev^T B X_new) is the projected start only for a B-orthonormal
  // X_prev; after the first step X_prev is the raw start block, and the start
  // it gives is still better than zero (a cold second step costs more Krylov
  // iterations), so every step's solutions are kept
  for (size_t q = 0; q < act.size(); ++q) act[q]->has_prev = st == SLRF_OK && fj[q].yprev != nullptr;
  if (st == SLRF_OK) st = finish_outer_all(env, act, fj);
  if (st != SLRF_OK)
    for (SolveJob* J : act)
      if (!J->done) {
        J->done = true;
        J->status = st;
        J->msg = env.err;
        J->ss.outer_iterations = J->k;
        J->ss.seconds = now_s() - J->t0;
      }
  return st;
}

slrf_status prepare_job(Env& env, SolveJob& J, double gamma, const slrf_poles* poles_in, const double* d_V0,
                        int max_N) {
  J.gamma = gamma;
  const slrf_poles* poles = poles_in;
  slrf_poles designed{};
  std::vector<double> ds, dw;
  if (!poles) {
    ds.resize(2 * kDefaultPoles);
    dw.resize(2 * kDefaultPoles);
    if (slrf_design_poles(kDefaultPoles, 1.0, 0.01, gamma, ds.data(), dw.data(), nullptr) != SLRF_OK)
      return fail(env, SLRF_E_INVALID_ARG, "pole design failed");
    designed = {kDefaultPoles, ds.data(), dw.data()};
    poles = &designed;
  }
  slrf_status st = check_poles(env, poles, max_N);
  if (st != SLRF_OK) return st;
  J.N = poles->n_poles;
  J.sig.assign(poles->sigma, poles->sigma + 2 * J.N);
  J.w.assign(poles->weight, poles->weight + 2 * J.N);
  J.t0 = now_s();
  if (d_V0)
    HIPCHK(env, hipMemcpyAsync(J.V, d_V0, 8 * (size_t)J.P->n * J.L, hipMemcpyDeviceToDevice, env.stream));
  else
    launch_gaussian(env.stream, (int64_t)J.P->n * J.L, env.opt.seed, J.V);
  HIPCHK(env, hipGetLastError());
  HIPCHK(env, hipStreamSynchronize(env.stream));
  return SLRF_OK;
}

slrf_status copy_results(Env& env, const SolveJob& J, int64_t* n_found, double* h_evals, double* d_evecs,
                         double* h_resid, slrf_solve_stats* stats) {
  HIPCHK(env, hipMemcpyAsync(d_evecs, J.V, 8 * (size_t)J.P->n * J.L, hipMemcpyDeviceToDevice, env.stream));
  HIPCHK(env, hipStreamSynchronize(env.stream));
  for (int c = 0; c < J.L; ++c) {
    h_evals[c] = c < (int)J.theta.size() ? J.theta[c] : 0.0;
    h_resid[c] = c < (int)J.rho.size() ? J.rho[c] : 0.0;
  }
  *n_found = J.ss.n_found;
  if (stats) *stats = J.ss;
  return SLRF_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Single-pencil context: [pencil | timer counters | filter arena | outer buffers]

struct slrf_ctx_s {
  Env env;
  Pencil P;
  char* ws = nullptr;
  int64_t max_L = 0;
  int32_t max_N = 0;
  size_t arena_off = 0, arena_bytes = 0, outer_off = 0;
  int static_dev = -1;  // device whose static scratch this context holds (slrf_create_static)
};

// ---- static scratch for callers that cannot allocate ---------------------------
//
// slrf_create_static runs a context inside this file-scope array instead of a
// caller workspace.  Each device the library runs on holds its own copy until
// the process ends.  Host code never uses the array's name as an address: the
// device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and kept in g_scratch_ptr.  One context at a time may hold a
// device's array; the library clears whatever it needs zeroed on every call, so
// what an earlier context left there does not matter.
static __device__ __align__(256) unsigned char scratch[SLRF_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_held[kMaxDevices] = {};
}  // namespace

// Batch of pencils: [timer counters | filter arena | pool of pencils and outer buffers]
struct slrf_batch_s {
  Env env;
  Pool pool;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int max_N = 0;
  int next_id = 0;
  struct Entry {
    std::unique_ptr<Pencil> P;
    std::unique_ptr<SolveJob> J;
  };
  std::map<int, Entry> entries;

  std::vector<JobShape> active_shapes() const {
    std::vector<JobShape> js;
    for (const auto& kv : entries)
      if (!kv.second.J->done)
        js.push_back({kv.second.P->n, kv.second.P->nnz, kv.second.J->L, kv.second.J->N, kv.second.P->use_ilu, false,
                      kv.second.P->use_bjac, kv.second.P->sgs});
    return js;
  }
};

extern "C" {

void slrf_default_options(slrf_options* o) {
  if (!o) return;
  o->precision = SLRF_FP64;
  o->inner_tol = 1e-13;  // Section 4.2: BiCGStab stopping tolerance of the eigensolver runs
  o->inner_maxit = 1000;
  o->outer_tol = 1e-8;
  o->outer_maxit = 40;
  o->check_every = 10;
  o->seed = 1;
  o->precond = 0;
  o->profile = 0;
  o->graph = 0;
  o->tile_rows = 0;
  o->tile_wgs = 0;
  o->band_rows = 0;
  o->tune = 0;
  o->solver = 0;
  o->recycle = 0;
  o->sgs_omega = 0.0;  // by block size: kSgsOmegaNode for node blocks, 1 for points
}

const char* slrf_status_string(slrf_status s) {
  switch (s) {
    case SLRF_OK: return "ok";
    case SLRF_E_INVALID_ARG: return "invalid argument";
    case SLRF_E_NOT_SPD: return "A or B has a non-positive or missing diagonal entry";
    case SLRF_E_WORKSPACE: return "workspace too small or misaligned";
    case SLRF_E_DEVICE: return "HIP runtime error";
    case SLRF_E_NOT_CONVERGED: return "outer iteration did not converge";
    case SLRF_E_SUBSPACE_TOO_SMALL: return "subspace too small: every Ritz value lies in the interval";
    case SLRF_E_BREAKDOWN: return "breakdown of the projected problem";
  }
  return "unknown status";
}

const char* slrf_last_error(slrf_ctx ctx) { return ctx ? ctx->env.err.c_str() : "null context"; }

slrf_status slrf_design_poles(int32_t N, double alpha, double beta, double gamma, double* sigma_out,
                              double* weight_out, double* sep_out) {
  if (N < 1 || N > 16 || !(alpha > 0) || !(beta > 0) || !(gamma > 0) || !sigma_out || !weight_out)
    return SLRF_E_INVALID_ARG;
  std::vector<double> u;
  if (!design_unit_cached(N, alpha, beta, u)) return SLRF_E_INVALID_ARG;
  std::complex<double> dphi = 0;
  for (int j = 0; j < N; ++j) {
    const std::complex<double> sg(gamma * u[j], gamma * u[j] * alpha);
    const std::complex<double> wj(gamma * u[N + 2 * j], gamma * u[N + 2 * j + 1]);
    sigma_out[2 * j] = sg.real();
    sigma_out[2 * j + 1] = sg.imag();
    weight_out[2 * j] = wj.real();
    weight_out[2 * j + 1] = wj.imag();
    dphi += -2.0 * (wj / ((gamma - sg) * (gamma - sg))).real();
  }
  if (sep_out) *sep_out = std::abs(dphi.real());
  return SLRF_OK;
}

slrf_status slrf_quadrature_poles(int32_t rule, int32_t N, double gamma, double* sigma_out, double* weight_out) {
  if (!sigma_out || !weight_out || !quadrature_poles(rule, N, gamma, sigma_out, weight_out))
    return SLRF_E_INVALID_ARG;
  return SLRF_OK;
}

slrf_status slrf_workspace_bytes_for(int64_t n, int64_t nnz, int64_t L, int32_t N, const slrf_options* opt,
                                     size_t* bytes) {
  slrf_options o;
  if (opt)
    o = *opt;
  else
    slrf_default_options(&o);
  if (n < 1 || nnz < n || L < 1 || N < 1 || !bytes || n > INT32_MAX || nnz > INT32_MAX) return SLRF_E_INVALID_ARG;
  if (o.precision != SLRF_FP64 && o.precision != SLRF_MIXED) return SLRF_E_INVALID_ARG;
  if (o.precond < 0 || o.precond > 5) return SLRF_E_INVALID_ARG;
  if (o.sgs_omega != 0.0 && !(o.sgs_omega > 0.0 && o.sgs_omega < 2.0)) return SLRF_E_INVALID_ARG;
  if (sgs_block_for(o.precond) && o.solver != 1) return SLRF_E_INVALID_ARG;
  if (o.solver == 1 && o.precond == 0) o.precond = 1;  // COCG runs with point Jacobi
  const size_t arena = filter_arena_bytes(
      {JobShape{n, nnz, (int)L, (int)N, use_ilu_for(o.precond, n, nnz), false, use_bjac_for(o.precond),
                sgs_block_for(o.precond)}},
      o.precision == SLRF_MIXED);
  *bytes = pencil_bytes(n, nnz, o.precond) + al(kTimerSlots * 4) + arena +
           outer_bytes(n, L, N, o.recycle && o.precision == SLRF_MIXED);
  return SLRF_OK;
}

slrf_status slrf_workspace_bytes(int64_t n, int64_t nnz, int64_t L, int32_t N, int32_t precision, size_t* bytes) {
  slrf_options o;
  slrf_default_options(&o);  // automatic preconditioner choice
  o.precision = precision;
  return slrf_workspace_bytes_for(n, nnz, L, N, &o, bytes);
}

slrf_status slrf_create_static(slrf_ctx* out, int64_t n, const int32_t* a_rowptr, const int32_t* a_col,
                               const double* a_val, const int32_t* b_rowptr, const int32_t* b_col,
                               const double* b_val, int64_t max_L, int32_t max_N, const slrf_options* opt,
                               void* hip_stream) {
  if (!out) return SLRF_E_INVALID_ARG;
  *out = nullptr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SLRF_E_DEVICE;
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SLRF_E_DEVICE;
      g_scratch_ptr[dev] = ptr;
    }
    ptr = g_scratch_ptr[dev];
    if (g_scratch_held[dev]) {
      slrf_ctx c = new (std::nothrow) slrf_ctx_s();
      if (!c) return SLRF_E_WORKSPACE;
      c->env.err = "the static scratch of device " + std::to_string(dev) + " is held by another context";
      *out = c;
      return SLRF_E_WORKSPACE;
    }
    g_scratch_held[dev] = true;
  }
  const slrf_status st = slrf_create(out, n, a_rowptr, a_col, a_val, b_rowptr, b_col, b_val, ptr,
                                     SLRF_STATIC_SCRATCH_BYTES, max_L, max_N, opt, hip_stream);
  if (*out) {
    (*out)->static_dev = dev;  // released by slrf_destroy, also after a failed create
  } else {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    g_scratch_held[dev] = false;
  }
  return st;
}

slrf_status slrf_create(slrf_ctx* out, int64_t n, const int32_t* a_rowptr, const int32_t* a_col,
                        const double* a_val, const int32_t* b_rowptr, const int32_t* b_col, const double* b_val,
                        void* d_workspace, size_t ws_bytes, int64_t max_L, int32_t max_N, const slrf_options* opt,
                        void* hip_stream) {
  if (!out) return SLRF_E_INVALID_ARG;
  *out = nullptr;
  slrf_ctx ctx = new (std::nothrow) slrf_ctx_s();
  if (!ctx) return SLRF_E_INVALID_ARG;
  *out = ctx;  // kept on failure so the caller can read the message
  Env& env = ctx->env;
  slrf_status st = setup_env(env, opt, hip_stream);
  if (st != SLRF_OK) return st;
  if (max_L < 1 || max_N < 1) return fail(env, SLRF_E_INVALID_ARG, "bad size or NULL argument");
  int64_t nnz = 0;
  st = build_pencil(n, a_rowptr, a_col, a_val, b_rowptr, b_col, b_val, env.opt.precond, env.opt.band_rows, env.stream, ctx->P, env.err,
                    nullptr, &nnz);
  if (st != SLRF_OK) return st;
  if (!d_workspace || ((uintptr_t)d_workspace & 255) != 0)
    return fail(env, SLRF_E_WORKSPACE, "workspace NULL or not 256-byte aligned");
  size_t need = 0;
  if (slrf_workspace_bytes_for(n, nnz, max_L, max_N, &env.opt, &need) != SLRF_OK)
    return fail(env, SLRF_E_INVALID_ARG, "bad sizes");
  if (ws_bytes < need)
    return fail(env, SLRF_E_WORKSPACE,
                "workspace has " + std::to_string(ws_bytes) + " bytes, needs " + std::to_string(need));
  ctx->max_L = max_L;
  ctx->max_N = max_N;
  st = build_pencil(n, a_rowptr, a_col, a_val, b_rowptr, b_col, b_val, env.opt.precond, env.opt.band_rows, env.stream, ctx->P, env.err,
                    (char*)d_workspace, nullptr);
  if (st != SLRF_OK) return st;
  const size_t poff = pencil_bytes(n, nnz, env.opt.precond);
  if (!env.setup_timer((int*)((char*)d_workspace + poff))) return fail(env, SLRF_E_DEVICE, "timer set-up failed");
  ctx->arena_off = poff + al(kTimerSlots * 4);
  ctx->arena_bytes =
      filter_arena_bytes({JobShape{n, nnz, (int)max_L, max_N, ctx->P.use_ilu, false, ctx->P.use_bjac, ctx->P.sgs}},
                         env.opt.precision == SLRF_MIXED);
  ctx->outer_off = ctx->arena_off + ctx->arena_bytes;
  ctx->ws = (char*)d_workspace;
  return SLRF_OK;
}

void slrf_destroy(slrf_ctx ctx) {
  if (!ctx) return;
  if (ctx->static_dev >= 0) {
    // work queued in the static scratch must finish before another context may use it
    (void)hipStreamSynchronize(ctx->env.stream);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    g_scratch_held[ctx->static_dev] = false;
  }
  delete ctx;
}

slrf_status slrf_filter_apply(slrf_ctx ctx, const slrf_poles* poles, int64_t L, const double* d_X, double* d_U,
                              slrf_filter_stats* stats) {
  if (!ctx || !ctx->ws) return SLRF_E_INVALID_ARG;
  Env& env = ctx->env;
  if (L < 1 || L > ctx->max_L || !d_X || !d_U || d_X == d_U)
    return fail(env, SLRF_E_INVALID_ARG, "bad L or block pointers");
  slrf_status st = check_poles(env, poles, ctx->max_N);
  if (st != SLRF_OK) return st;
  std::vector<FilterJob> jobs{
      {&ctx->P, (int)L, poles->n_poles, poles->sigma, poles->weight, d_X, d_U, env.opt.inner_tol, {}}};
  Carver arena{ctx->ws + ctx->arena_off, 0, ctx->arena_bytes};
  st = filter_batch(env, arena, jobs);
  if (st != SLRF_OK) return st;
  if (stats) *stats = jobs[0].stats;
  return SLRF_OK;
}

slrf_status slrf_solve_interval(slrf_ctx ctx, double gamma, int64_t L, const slrf_poles* poles, const double* d_V0,
                                int64_t* n_found, double* h_evals, double* d_evecs, double* h_resid,
                                slrf_solve_stats* stats) {
  if (!ctx || !ctx->ws) return SLRF_E_INVALID_ARG;
  Env& env = ctx->env;
  if (!(gamma > 0) || L < 2 || L > ctx->max_L || !n_found || !h_evals || !d_evecs || !h_resid)
    return fail(env, SLRF_E_INVALID_ARG, "bad gamma, L or output pointer");
  if (L > ctx->P.n) return fail(env, SLRF_E_INVALID_ARG, "L exceeds n");
  SolveJob J;
  J.P = &ctx->P;
  J.L = (int)L;
  J.carve(ctx->ws + ctx->outer_off, ctx->max_N, env.opt.recycle && env.opt.precision == SLRF_MIXED);
  slrf_status st = prepare_job(env, J, gamma, poles, d_V0, ctx->max_N);
  if (st != SLRF_OK) return st;
  const std::vector<SolveJob*> jobs{&J};
  while (!J.done) {
    st = outer_step(env, Carver{ctx->ws + ctx->arena_off, 0, ctx->arena_bytes}, jobs);
    if (st != SLRF_OK) return st;
  }
  st = copy_results(env, J, n_found, h_evals, d_evecs, h_resid, stats);
  if (st != SLRF_OK) return st;
  if (J.status != SLRF_OK) return fail(env, J.status, J.msg);
  return SLRF_OK;
}

// ---- batches ------------------------------------------------------------------

slrf_status slrf_batch_footprint_for(int64_t n, int64_t nnz, int64_t L, int32_t N, const slrf_options* opt,
                                     size_t* persistent_bytes, size_t* transient_bytes) {
  slrf_options o;
  if (opt)
    o = *opt;
  else
    slrf_default_options(&o);
  if (n < 1 || nnz < n || L < 1 || N < 1 || n > INT32_MAX || nnz > INT32_MAX || !persistent_bytes ||
      !transient_bytes)
    return SLRF_E_INVALID_ARG;
  if (o.precision != SLRF_FP64 && o.precision != SLRF_MIXED) return SLRF_E_INVALID_ARG;
  if (o.precond < 0 || o.precond > 5) return SLRF_E_INVALID_ARG;
  if (o.sgs_omega != 0.0 && !(o.sgs_omega > 0.0 && o.sgs_omega < 2.0)) return SLRF_E_INVALID_ARG;
  const int sgs = sgs_block_for(o.precond);
  // with room for the warm-start blocks (options.recycle) in mixed precision
  *persistent_bytes = al(pencil_bytes(n, nnz, o.precond)) + al(outer_bytes(n, L, N, o.precision == SLRF_MIXED));
  // counts the two blocks a batch with an ILU(0) or block-Jacobi pencil gives
  // every pencil (and block-Jacobi inverses when n is a multiple of 3), so that
  // the sum over a set of pencils bounds the arena the set needs
  *transient_bytes = filter_arena_bytes(
      {JobShape{n, nnz, (int)L, (int)N, ilu_allowed(n, nnz), true, n % 3 == 0, sgs}}, o.precision == SLRF_MIXED);
  return SLRF_OK;
}

slrf_status slrf_batch_footprint(int64_t n, int64_t nnz, int64_t L, int32_t N, int32_t precision,
                                 size_t* persistent_bytes, size_t* transient_bytes) {
  slrf_options o;
  slrf_default_options(&o);
  o.precision = precision;
  return slrf_batch_footprint_for(n, nnz, L, N, &o, persistent_bytes, transient_bytes);
}

const char* slrf_batch_last_error(slrf_batch b) { return b ? b->env.err.c_str() : "null batch"; }

slrf_status slrf_batch_create(slrf_batch* out, void* d_workspace, size_t ws_bytes, size_t arena_bytes,
                              int32_t max_poles, const slrf_options* opt, void* hip_stream) {
  if (!out) return SLRF_E_INVALID_ARG;
  *out = nullptr;
  slrf_batch b = new (std::nothrow) slrf_batch_s();
  if (!b) return SLRF_E_INVALID_ARG;
  *out = b;
  Env& env = b->env;
  slrf_status st = setup_env(env, opt, hip_stream);
  if (st != SLRF_OK) return st;
  if (max_poles < 1 || max_poles > 16) return fail(env, SLRF_E_INVALID_ARG, "max_poles must be in [1, 16]");
  if (!d_workspace || ((uintptr_t)d_workspace & 255) != 0)
    return fail(env, SLRF_E_WORKSPACE, "workspace NULL or not 256-byte aligned");
  const size_t head = al(kTimerSlots * 4);
  if (ws_bytes < head + al(arena_bytes))
    return fail(env, SLRF_E_WORKSPACE, "workspace smaller than the arena it should hold");
  char* ws = (char*)d_workspace;
  if (!env.setup_timer((int*)ws)) return fail(env, SLRF_E_DEVICE, "timer set-up failed");
  b->arena = ws + head;
  b->arena_bytes = al(arena_bytes);
  b->pool.init(ws + head + b->arena_bytes, ws_bytes - head - b->arena_bytes);
  b->max_N = max_poles;
  return SLRF_OK;
}

slrf_status slrf_batch_add(slrf_batch b, int64_t n, const int32_t* a_rowptr, const int32_t* a_col,
                           const double* a_val, const int32_t* b_rowptr, const int32_t* b_col, const double* b_val,
                           double gamma, int64_t L, const slrf_poles* poles, const double* d_V0, int32_t* id) {
  if (!b || !id) return SLRF_E_INVALID_ARG;
  Env& env = b->env;
  if (!(gamma > 0) || L < 2 || L > n || L > INT32_MAX) return fail(env, SLRF_E_INVALID_ARG, "bad gamma or L");
  const int N = poles ? poles->n_poles : kDefaultPoles;
  if (N < 1 || N > b->max_N) return fail(env, SLRF_E_INVALID_ARG, "pole count outside [1, max_poles]");
  int64_t nnz = 0;
  auto P = std::make_unique<Pencil>();
  slrf_status st = build_pencil(n, a_rowptr, a_col, a_val, b_rowptr, b_col, b_val, env.opt.precond, env.opt.band_rows, env.stream, *P,
                                env.err, nullptr, &nnz);
  if (st != SLRF_OK) return st;
  std::vector<JobShape> shapes = b->active_shapes();
  shapes.push_back({n, nnz, (int)L, N, use_ilu_for(env.opt.precond, n, nnz), false, use_bjac_for(env.opt.precond),
                    sgs_block_for(env.opt.precond)});
  if (filter_arena_bytes(shapes, env.opt.precision == SLRF_MIXED) > b->arena_bytes)
    return fail(env, SLRF_E_WORKSPACE, "the filter arena cannot hold this pencil next to the active ones");
  const bool warm = env.opt.recycle && env.opt.precision == SLRF_MIXED;
  const size_t pb = pencil_bytes(n, nnz, env.opt.precond), ob = outer_bytes(n, L, N, warm);
  char* pm = b->pool.alloc(pb);
  if (!pm) return fail(env, SLRF_E_WORKSPACE, "no room for the pencil in the workspace");
  char* om = b->pool.alloc(ob);
  if (!om) {
    b->pool.release(pm, pb);
    return fail(env, SLRF_E_WORKSPACE, "no room for the subspace blocks in the workspace");
  }
  auto J = std::make_unique<SolveJob>();
  st = build_pencil(n, a_rowptr, a_col, a_val, b_rowptr, b_col, b_val, env.opt.precond, env.opt.band_rows, env.stream, *P, env.err, pm,
                    nullptr);
  if (st == SLRF_OK) {
    J->P = P.get();
    J->L = (int)L;
    J->carve(om, N, warm);
    st = prepare_job(env, *J, gamma, poles, d_V0, b->max_N);
  }
  if (st != SLRF_OK) {
    b->pool.release(pm, pb);
    b->pool.release(om, ob);
    return st;
  }
  *id = b->next_id++;
  b->entries[*id] = {std::move(P), std::move(J)};
  return SLRF_OK;
}

slrf_status slrf_batch_step(slrf_batch b, int32_t* n_active) {
  if (!b) return SLRF_E_INVALID_ARG;
  std::vector<SolveJob*> jobs;
  for (auto& kv : b->entries)
    if (!kv.second.J->done) jobs.push_back(kv.second.J.get());
  const slrf_status st = outer_step(b->env, Carver{b->arena, 0, b->arena_bytes}, jobs);
  int act = 0;
  for (auto& kv : b->entries)
    if (!kv.second.J->done) ++act;
  if (n_active) *n_active = act;
  return st;
}

slrf_status slrf_batch_query(slrf_batch b, int32_t id, int32_t* done, int32_t* outer_iterations) {
  if (!b) return SLRF_E_INVALID_ARG;
  auto it = b->entries.find(id);
  if (it == b->entries.end()) return fail(b->env, SLRF_E_INVALID_ARG, "unknown pencil id");
  if (done) *done = it->second.J->done ? 1 : 0;
  if (outer_iterations) *outer_iterations = it->second.J->k;
  return SLRF_OK;
}

slrf_status slrf_batch_result(slrf_batch b, int32_t id, int64_t* n_found, double* h_evals, double* d_evecs,
                              double* h_resid, slrf_solve_stats* stats) {
  if (!b) return SLRF_E_INVALID_ARG;
  if (!n_found || !h_evals || !d_evecs || !h_resid) return fail(b->env, SLRF_E_INVALID_ARG, "NULL output pointer");
  auto it = b->entries.find(id);
  if (it == b->entries.end()) return fail(b->env, SLRF_E_INVALID_ARG, "unknown pencil id");
  const SolveJob& J = *it->second.J;
  if (!J.done) return fail(b->env, SLRF_E_INVALID_ARG, "pencil not finished");
  slrf_status st = copy_results(b->env, J, n_found, h_evals, d_evecs, h_resid, stats);
  if (st != SLRF_OK) return st;
  if (J.status != SLRF_OK) return fail(b->env, J.status, J.msg);
  return SLRF_OK;
}

slrf_status slrf_batch_restart(slrf_batch b, int32_t id, const double* d_V0) {
  if (!b) return SLRF_E_INVALID_ARG;
  auto it = b->entries.find(id);
  if (it == b->entries.end()) return fail(b->env, SLRF_E_INVALID_ARG, "unknown pencil id");
  Env& env = b->env;
  const SolveJob& old = *it->second.J;
  auto J = std::make_unique<SolveJob>();
  J->P = old.P;
  J->L = old.L;
  // the same device buffers, sized for the batch's max_N at add
  J->carve(old.mem, b->max_N, env.opt.recycle && env.opt.precision == SLRF_MIXED);
  const slrf_poles poles{old.N, old.sig.data(), old.w.data()};
  const slrf_status st = prepare_job(env, *J, old.gamma, &poles, d_V0, b->max_N);
  if (st != SLRF_OK) return st;
  it->second.J = std::move(J);
  return SLRF_OK;
}

slrf_status slrf_batch_remove(slrf_batch b, int32_t id) {
  if (!b) return SLRF_E_INVALID_ARG;
  auto it = b->entries.find(id);
  if (it == b->entries.end()) return fail(b->env, SLRF_E_INVALID_ARG, "unknown pencil id");
  const Pencil& P = *it->second.P;
  const SolveJob& J = *it->second.J;
  b->pool.release(P.mem, P.mem_bytes);
  b->pool.release(J.mem, J.mem_bytes);
  b->entries.erase(it);
  return SLRF_OK;
}

void slrf_batch_destroy(slrf_batch b) { delete b; }

// ---- kernel-level test hooks ----------------------------------------------

size_t slrf_test_gram_scratch(int64_t n, int64_t L) {
  return (size_t)gram_chunks((int)n, (int)L) * 2 * L * L * sizeof(double);
}

int slrf_test_gram(int64_t n, int64_t L, const double* U, const double* WA, const double* WB, double* GA,
                   double* GB, void* scratch, size_t scratch_bytes, void* hip_stream) {
  return slrf_test_gram_prec(n, L, U, WA, WB, GA, GB, scratch, scratch_bytes, 0, hip_stream);
}

int slrf_test_gram_prec(int64_t n, int64_t L, const double* U, const double* WA, const double* WB, double* GA,
                        double* GB, void* scratch, size_t scratch_bytes, int f32, void* hip_stream) {
  if (n < 1 || L < 1 || !U || !WA || !WB || !GA || !GB || scratch_bytes < slrf_test_gram_scratch(n, L))
    return SLRF_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)hip_stream;
  launch_gram(s, (int)n, (int)L, U, WA, WB, (double*)scratch, gram_chunks((int)n, (int)L), GA, GB, f32 != 0);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return SLRF_E_DEVICE;
  return SLRF_OK;
}

int slrf_test_gemm(int64_t n, int64_t L, int64_t r, const double* X, const double* Z, double* Y,
                   void* hip_stream) {
  if (n < 1 || L < 1 || r < 1 || !X || !Z || !Y) return SLRF_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)hip_stream;
  const double* xs[1] = {X};
  double* ys[1] = {Y};
  launch_gemm_nz(s, (int)n, (int)L, (int)r, 1, xs, Z, ys);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return SLRF_E_DEVICE;
  return SLRF_OK;
}

}  // extern "C"
