// Host side of the block-SR library: planner (validation, block layout, form
// and precision per block, workspace layout, work lists), executor (the kernel
// sequence of the form and solve steps) and the C ABI declared in qgt_block.h.
//
// Paper, Sec. 2: the parameters are split into disjoint layer groups, each
// block S_l of the QGT is shifted by a uniform lambda and inverted
// independently, and the block updates are concatenated in parameter order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/qgt_block.h"
#include "../../include/qgt_jacobian.h"
#include "qgt_internal.h"
#include "qgt_launch.h"

using namespace qgt;

namespace {

thread_local std::string g_last_error;

qgt_status fail(qgt_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

struct Layout {
  size_t bytes = 0;
  int64_t take(size_t n) {
    const int64_t off = (int64_t)round_up((int64_t)bytes, 256);
    bytes = (size_t)off + n;
    return off;
  }
};

struct TimingPair {
  hipEvent_t a = nullptr, b = nullptr;
  bool pending = false;
};

}  // namespace

struct qgt_plan_s {
  int nprob = 0;
  int dt = 0;
  int max_refine = 0;
  std::vector<ProbDev> probs;
  std::vector<BlockDev> blocks;
  std::vector<int32_t> user_forms;
  std::vector<qgt_block_tuning> tuning;             // per block, defaults filled in
  std::vector<int32_t> tuning_src;                  // 0 defaults, 1 caller, 2 tuning cache

  // work lists (host copies; device copies live in dmeta)
  std::vector<ColTile> col_all, col_s;
  std::vector<RowItem> row_p, row_s;
  std::vector<int32_t> gl_sorted, gl_p, gl_s;
  std::vector<int32_t> gl_pack[2][3];
  int64_t pack_maxmt[2][3] = {};
  int pack_ygrid[2][3] = {};
  std::vector<GramItem> gram_items[5];               // per precision (FP64, FP32, BF16), wide BF16, duo BF16
  int32_t gram_xcd[5][16] = {};                    // per list: 8 chunk starts, 8 chunk lengths
  int gram_maxlen[5] = {};
  std::vector<SplitItem> split_items;
  std::vector<int2> tmap_fwd, tmap_bwd;             // ticket -> (block, tile) of the triangular solves
  std::vector<int32_t> chol_count;                  // per step k: blocks with ntiles > k (prefix of gl_sorted)
  std::vector<int4> trsm_tasks, upd_tasks;          // (block, i, j, 0) per step, concatenated
  std::vector<int32_t> trsm_off;                    // per step k, size Tmax + 1
  std::vector<int32_t> upd_off;                     // per pair p: first single-step task, size Tmax/2 + 1
  std::vector<int32_t> upd_col;                     // per pair p: first K=128 task of columns k+2, k+3
  std::vector<int32_t> upd_mid;                     // per pair p: first K=128 task of the rest (j >= k+4)
  hipStream_t side = nullptr;                       // lookahead stream for the bulk of the updates
  int n_cu = 256;                                   // compute units of the plan's device
  int device = -1;                                  // the device the plan's metadata lives on
  hipEvent_t ev_main = nullptr, ev_side = nullptr;
  std::vector<CholTask> chol_tasks;                 // tile tasks of the persistent Cholesky, in priority order
  std::vector<CholTask> chol_qtasks;                // the same split into one ticket queue per XCD
  std::vector<int32_t> chol_qoff;                   // queue q: chol_qtasks[chol_qoff[q] .. chol_qoff[q + 1])
  int chol_nq = 1;                                  // queues (XCDs of the device)
  int chol_state_n = 0;                             // tile counters over all blocks
  bool chol_host_steps = false;                     // host-sequenced launches instead of the persistent one
  int32_t chol_mode_src = 0;                        // how that was chosen: 0 default, 1 caller, 2 tuning cache
  std::vector<int32_t> tile_base;                   // first tile of each block (host order check)
  int total_tiles = 0;
  int Tmax = 0;
  int RC = 1;
  int64_t max_mpad = 0, max_nb = 0;
  double gram_flops[3] = {0.0, 0.0, 0.0};  // algorithmic flops of one Gram launch, per precision

  // workspace layout
  size_t ws_bytes = 0;
  int64_t ptrs_off = 0, status_off = 0, floor_off = 0, bscal_off = 0, colpart_off = 0, gpart_off = 0, sync_off = 0, trace_off = 0;
  int64_t cg_off = 0, chol_state_off = 0, chol_ctl_off = 0;
  double rtol = 0.0;
  int sync_ints = 0;

  // device metadata
  char* dmeta = nullptr;
  int64_t m_probs = 0, m_blocks = 0, m_col_all = 0, m_col_s = 0, m_row_p = 0, m_row_s = 0, m_gl_sorted = 0,
          m_gl_p = 0, m_gl_s = 0, m_gl_pack[2][3] = {}, m_gram[5] = {}, m_gram_xcd[5] = {}, m_split = 0,
          m_tmap_fwd = 0, m_tmap_bwd = 0, m_trsm = 0, m_upd = 0, m_chol = 0, m_chol_qoff = 0;

  // bound per call
  char* ws = nullptr;
  BindArgs bind{};
  bool formed = false;

  // timing
  bool timing = false;
  std::vector<TimingPair> tpairs[3];  // event pairs around the Gram launch of each precision
  size_t tnext[3] = {0, 0, 0};
  double t_total_ms[3] = {0.0, 0.0, 0.0};
  int64_t t_launches[3] = {0, 0, 0};

  ~qgt_plan_s() {
    if (side) (void)hipStreamDestroy(side);
    if (ev_main) (void)hipEventDestroy(ev_main);
    if (ev_side) (void)hipEventDestroy(ev_side);
    if (dmeta) (void)hipFree(dmeta);
    for (auto& ring : tpairs)
      for (auto& p : ring) {
        if (p.a) (void)hipEventDestroy(p.a);
        if (p.b) (void)hipEventDestroy(p.b);
      }
  }

  template <typename T>
  const T* dev(int64_t off) const { return reinterpret_cast<const T*>(dmeta + off); }
  bool has_gram(int pr) const {
    return !gram_items[pr].empty() || (pr == PREC_BF16 && (!gram_items[3].empty() || !gram_items[4].empty()));
  }
};

namespace {

// ---------------------------------------------------------------------------
// Tuning: per-block tile shapes and schedules, from the caller, from the
// JSON cache the autotuner writes (QGT_TUNE_CACHE), or the defaults.
// ---------------------------------------------------------------------------
const char* prec_name(int prec) { return prec == PREC_FP64 ? "fp64" : (prec == PREC_FP32 ? "fp32" : "bf16"); }

bool wide_eligible(const BlockDev& bd) { return bd.prec == PREC_BF16 && bd.m_pad % 256 == 0 && bd.m_pad >= 1024; }

// Shape class of a block: everything the tuned launches depend on.  The
// library's code object is built for gfx950 only, so that is the arch.
std::string tune_class(const BlockDev& bd) {
  int64_t k = 1;
  while (k < bd.K_pad) k <<= 1;
  return std::string("gfx950/") + prec_name(bd.prec) + "/" + (bd.form == FORM_P ? "P" : "S") + "/m" +
         std::to_string(bd.m_pad) + "/k" + std::to_string(k) + (bd.fact32 ? "/f32" : "");
}

// Integer field `name` on a line of the cache ("name": value), or 0.
int32_t tune_field(const std::string& line, const char* name) {
  const std::string key = std::string("\"") + name + "\":";
  const size_t at = line.find(key);
  if (at == std::string::npos) return 0;
  return (int32_t)std::strtol(line.c_str() + at + key.size(), nullptr, 10);
}

// The cache: one entry per line, "class": {"gram_tile": .., ...} for a
// block's shape class, "plan class": {"cholesky": ..} for the launch mode of
// the Cholesky of a whole set of blocks, and "plan class/class" (the shape
// class without its arch) for the tuning of that class inside that set of
// blocks.  The last is what the autotuner measured for the set: the blocks of
// a set share their launches, so the best tiles of a class depend on the
// other blocks, and a set tuned in its own right keeps its choice when
// another set with the same class re-tunes the class entry.  Missing or
// unreadable files give an empty cache (the planner then uses defaults).
struct TuneCache {
  std::map<std::string, qgt_block_tuning> blocks;
  std::map<std::string, int32_t> plans;  // qgt_cholesky
  bool empty() const { return blocks.empty() && plans.empty(); }
};

// Class of a whole plan, for its Cholesky launch mode: the shape classes of
// all its blocks, sorted, hashed (FNV-1a, 64 bits), with the block count.
std::string plan_class(const std::vector<BlockDev>& blocks) {
  std::vector<std::string> keys;
  for (const BlockDev& bd : blocks) keys.push_back(tune_class(bd));
  std::sort(keys.begin(), keys.end());
  uint64_t h = 1469598103934665603ull;
  for (const std::string& k : keys) {
    for (unsigned char ch : k) h = (h ^ ch) * 1099511628211ull;
    h = (h ^ (unsigned char)'|') * 1099511628211ull;
  }
  char buf[64];
  std::snprintf(buf, sizeof buf, "gfx950/plan/%016llx/n%zu", (unsigned long long)h, blocks.size());
  return buf;
}

// Key of a shape class inside a plan class: "gfx950/plan/<hash>/n<count>/"
// followed by the shape class without its "gfx950/".
std::string plan_block_key(const std::string& plan, const std::string& cls) {
  const size_t slash = cls.find('/');
  return plan + "/" + (slash == std::string::npos ? cls : cls.substr(slash + 1));
}

TuneCache read_tune_cache(const char* path, bool* ok) {
  TuneCache out;
  if (ok) *ok = true;
  FILE* f = path ? std::fopen(path, "r") : nullptr;
  if (!f) {
    if (ok) *ok = path == nullptr;
    return out;
  }
  char buf[4096];
  while (std::fgets(buf, sizeof buf, f)) {
    const std::string line(buf);
    const size_t q0 = line.find('"');
    const size_t q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
    if (q1 == std::string::npos) continue;
    if (line.find("\"cholesky\"") != std::string::npos) {
      out.plans[line.substr(q0 + 1, q1 - q0 - 1)] = tune_field(line, "cholesky");
      continue;
    }
    if (line.find("\"gram_tile\"") == std::string::npos) continue;
    qgt_block_tuning t{};
    t.gram_tile = tune_field(line, "gram_tile");
    t.gram_items = tune_field(line, "gram_items");
    t.chol_chunk = tune_field(line, "chol_chunk");
    t.gram_patch = tune_field(line, "gram_patch");
    out.blocks[line.substr(q0 + 1, q1 - q0 - 1)] = t;
  }
  std::fclose(f);
  return out;
}

// Fill in the defaults and check the ranges.
qgt_status resolve_tuning(const BlockDev& bd, qgt_block_tuning& t) {
  if (t.gram_tile == 0) t.gram_tile = wide_eligible(bd) ? 2 : 1;
  if (t.gram_items == 0) t.gram_items = 256;
  if (t.chol_chunk == 0) t.chol_chunk = 4;
  if (t.gram_patch == 0) t.gram_patch = 4;
  if (t.gram_tile != 1 && !(t.gram_tile == 2 && wide_eligible(bd)) && !(t.gram_tile == 3 && bd.prec == PREC_BF16))
    return fail(QGT_ERR_INVALID_ARGUMENT,
                "gram_tile must be 1, 2 for a BF16 block of order a multiple of 256 >= 1024, or 3 for a BF16 block");
  if (t.gram_items < 1 || t.gram_items > 65536) return fail(QGT_ERR_INVALID_ARGUMENT, "gram_items out of range");
  if (t.chol_chunk < 1 || t.chol_chunk > 16) return fail(QGT_ERR_INVALID_ARGUMENT, "chol_chunk must be in [1, 16]");
  if (t.gram_patch < 1 || t.gram_patch > 16) return fail(QGT_ERR_INVALID_ARGUMENT, "gram_patch must be in [1, 16]");
  return QGT_OK;
}

qgt_status validate(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype, qgt_precision gram,
                    int32_t max_refine, const qgt_plan_options* opts) {
  if (!probs) return fail(QGT_ERR_INVALID_ARGUMENT, "probs is null");
  if (n_probs < 1 || n_probs > kMaxProblems)
    return fail(QGT_ERR_INVALID_ARGUMENT, "n_probs must be in [1, " + std::to_string(kMaxProblems) + "]");
  if (o_dtype != QGT_C64 && o_dtype != QGT_C128) return fail(QGT_ERR_INVALID_ARGUMENT, "unknown O dtype");
  if (gram < QGT_GRAM_FP64 || gram > QGT_GRAM_AUTO) return fail(QGT_ERR_INVALID_ARGUMENT, "unknown Gram precision");
  if (max_refine < 0 || max_refine > 16) return fail(QGT_ERR_INVALID_ARGUMENT, "max_refine must be in [0, 16]");
  int64_t total_blocks = 0;
  for (int p = 0; p < n_probs; ++p) {
    const qgt_problem& q = probs[p];
    if (q.n_samples < 2) return fail(QGT_ERR_INVALID_ARGUMENT, "problem " + std::to_string(p) + ": n_samples < 2");
    if (q.n_samples > (int64_t)1 << 24)
      return fail(QGT_ERR_UNSUPPORTED, "problem " + std::to_string(p) + ": n_samples above 2^24");
    if (q.n_blocks < 1 || !q.block_sizes)
      return fail(QGT_ERR_INVALID_ARGUMENT, "problem " + std::to_string(p) + ": no blocks");
    if (!(q.lambda > 0.0) || !std::isfinite(q.lambda))
      return fail(QGT_ERR_INVALID_ARGUMENT, "problem " + std::to_string(p) + ": lambda must be positive and finite");
    int64_t np = 0;
    for (int b = 0; b < q.n_blocks; ++b) {
      if (q.block_sizes[b] < 1)
        return fail(QGT_ERR_INVALID_ARGUMENT, "problem " + std::to_string(p) + ": block size must be positive");
      np += q.block_sizes[b];
    }
    if (np > ((int64_t)1 << 31) - 1) return fail(QGT_ERR_UNSUPPORTED, "n_p above 2^31");
    total_blocks += q.n_blocks;
  }
  if (total_blocks > 65535) return fail(QGT_ERR_UNSUPPORTED, "more than 65535 blocks");
  if (opts && opts->factor != QGT_FACTOR_FP64 && opts->factor != QGT_FACTOR_FP32_FOR_BF16)
    return fail(QGT_ERR_INVALID_ARGUMENT, "unknown factor precision");
  if (opts && (opts->cholesky < QGT_CHOL_AUTO || opts->cholesky > QGT_CHOL_PERSISTENT))
    return fail(QGT_ERR_INVALID_ARGUMENT, "unknown Cholesky launch mode");
  if (opts && opts->forms) {
    for (int64_t g = 0; g < total_blocks; ++g)
      if (opts->forms[g] < QGT_FORM_AUTO || opts->forms[g] > QGT_FORM_SAMPLE)
        return fail(QGT_ERR_INVALID_ARGUMENT, "unknown form override");
  }
  return QGT_OK;
}

// Tile tasks of the Cholesky of one block (T tiles per side, update chunks of
// c panels) in column order, which is topological, with the bottom level of
// each task: the longest path from its start to the end of the block's
// factorisation, in rough microseconds per task kind (a 64x64 POTRF with its
// inverse; a 64x64x64 complex tile product).
void chol_block_tasks(int g, int T, int c, std::vector<CholTask>& tasks, std::vector<double>& bl) {
  tasks.clear();
  std::vector<int> first((size_t)T * (T + 1) / 2);
  for (int j = 0; j < T; ++j) {
    const int nch = chol_nchunks(j, c);
    for (int i = j; i < T; ++i) {
      first[(size_t)tri_index(i, j)] = (int)tasks.size();
      for (int u = 0; u < nch; ++u) {
        int k0 = 0, k1 = 0;
        chol_chunk_bounds(j, c, u, k0, k1);
        tasks.push_back(CholTask{g, CHOL_UPD, (int16_t)i, (int16_t)j, (int16_t)k0, (int16_t)k1, (int16_t)u});
      }
      tasks.push_back(
          CholTask{g, (int16_t)(i == j ? CHOL_POTRF : CHOL_TRSM), (int16_t)i, (int16_t)j, 0, 0, (int16_t)nch});
    }
  }
  auto final_op = [&](int a, int k) { return first[(size_t)tri_index(a, k)] + chol_nchunks(k, c); };
  const size_t n = tasks.size();
  std::vector<double> acc(n, 0.0);
  bl.assign(n, 0.0);
  for (size_t x = n; x-- > 0;) {
    const CholTask& t = tasks[x];
    const double dur = t.type == CHOL_POTRF ? 30.0 : (t.type == CHOL_TRSM ? 8.0 : 3.0 + 5.0 * (t.k1 - t.k0));
    bl[x] = dur + acc[x];
    auto relax = [&](int p) { acc[(size_t)p] = std::max(acc[(size_t)p], bl[x]); };
    if (t.seq > 0) relax(first[(size_t)tri_index(t.i, t.j)] + t.seq - 1);
    if (t.type == CHOL_UPD) {
      for (int k = t.k0; k < t.k1; ++k) {
        relax(final_op(t.i, k));
        relax(final_op(t.j, k));
      }
    } else if (t.type == CHOL_TRSM) {
      relax(final_op(t.j, t.j));
    }
  }
}

// The persistent Cholesky's tasks split into one ticket queue per XCD: every
// operation on tile (i, j) of block g goes to XCD chol_owner(g, i, j), so a
// tile's intermediate values are only ever read and written under that XCD's
// L2, and only final tiles cross XCDs.  Each queue keeps the global priority
// order (a subsequence of a topological order of every block's graph).
void split_chol_queues(qgt_plan_s& P, int nq) {
  P.chol_nq = nq;
  P.chol_qoff.assign(nq + 1, 0);
  std::vector<std::vector<CholTask>> q(nq);
  for (const CholTask& t : P.chol_tasks) q[chol_owner(t.g, t.i, t.j, nq)].push_back(t);
  P.chol_qtasks.clear();
  for (int x = 0; x < nq; ++x) {
    P.chol_qoff[x] = (int32_t)P.chol_qtasks.size();
    P.chol_qtasks.insert(P.chol_qtasks.end(), q[x].begin(), q[x].end());
  }
  P.chol_qoff[nq] = (int32_t)P.chol_qtasks.size();
}

// Build everything that does not need the GPU.
qgt_status build_plan(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype, qgt_precision gram,
                      int32_t max_refine, const qgt_plan_options* opts, qgt_plan_s& P, bool use_cache = true) {
  qgt_status st = validate(probs, n_probs, o_dtype, gram, max_refine, opts);
  if (st != QGT_OK) return st;
  P.nprob = n_probs;
  P.dt = o_dtype == QGT_C64 ? 0 : 1;
  P.max_refine = max_refine;
  P.timing = opts && opts->timing;
  Layout L;
  P.ptrs_off = L.take(sizeof(ProbPtrs) * kMaxProblems);

  int g = 0;
  for (int p = 0; p < n_probs; ++p) {
    const qgt_problem& q = probs[p];
    ProbDev pd{};
    pd.n_s = q.n_samples;
    pd.n_p = 0;
    for (int b = 0; b < q.n_blocks; ++b) pd.n_p += q.block_sizes[b];
    pd.first_block = g;
    pd.n_blocks = q.n_blocks;
    pd.lambda = q.lambda;
    pd.inv_ns = 1.0 / (double)q.n_samples;
    int64_t off = 0;
    for (int b = 0; b < q.n_blocks; ++b, ++g) {
      BlockDev bd{};
      bd.prob = p;
      bd.col_off = off;
      bd.n_b = q.block_sizes[b];
      off += bd.n_b;
      int form = (opts && opts->forms) ? opts->forms[g] : QGT_FORM_AUTO;
      if (form == QGT_FORM_AUTO) form = q.n_samples < bd.n_b ? QGT_FORM_SAMPLE : QGT_FORM_PARAM;
      bd.form = form == QGT_FORM_SAMPLE ? FORM_S : FORM_P;
      int prec = gram;
      // AUTO: FP64 for complex128 input.  For complex64 input the precision
      // follows how well the block is conditioned by its shape.  A Gram whose
      // operand is far from square (n_b >= 2 n_s in sample space) has its
      // smallest nonzero eigenvalues well away from zero and takes BF16; near
      // n_b = n_s the smallest eigenvalues approach zero and the block takes
      // FP32.  Parameter-space blocks can also have exact null directions
      // (first-layer weights under zero magnetisation) that a low-precision
      // Gram resolves poorly, so they take FP64 where that is affordable
      // (<= 1e11 flops, about two milliseconds on the FP64 matrix cores) and
      // FP32 otherwise.  The CG iteration removes the rounding in every case;
      // the choice sets how many iterations that takes.
      if (prec == QGT_GRAM_AUTO) {
        const double ns = (double)q.n_samples, nb = (double)bd.n_b;
        if (o_dtype == QGT_C128) prec = QGT_GRAM_FP64;
        else if (form == QGT_FORM_SAMPLE) prec = nb >= 2.0 * ns ? QGT_GRAM_BF16 : QGT_GRAM_FP32;
        else prec = 4.0 * ns * nb * nb <= 1e11 ? QGT_GRAM_FP64 : QGT_GRAM_FP32;
      }
      bd.prec = prec;
      bd.fact32 = (opts && opts->factor == QGT_FACTOR_FP32_FOR_BF16 && prec == QGT_GRAM_BF16) ? 1 : 0;
      bd.m = bd.form == FORM_P ? bd.n_b : q.n_samples;
      bd.K = bd.form == FORM_P ? q.n_samples : bd.n_b;
      bd.m_pad = round_up(bd.m, kGramTile);
      bd.K_pad = round_up(bd.K, gram_stage_k(prec));
      bd.ntiles = (int32_t)(bd.m_pad / kTile);
      bd.lambda = q.lambda;
      bd.inv_ns = pd.inv_ns;
      P.blocks.push_back(bd);
    }
    P.probs.push_back(pd);
  }
  const int nb = (int)P.blocks.size();
  // Tile shapes and schedules per block: the caller's, else the tuning
  // cache's entry for the block's shape class inside this set of blocks, else
  // its entry for the shape class, else the defaults.
  {
    TuneCache cache;
    const char* cache_path = use_cache ? std::getenv("QGT_TUNE_CACHE") : nullptr;
    if (cache_path && *cache_path) cache = read_tune_cache(cache_path, nullptr);
    if (opts && opts->tuning) cache.blocks.clear();  // the caller's tuning wins
    P.tuning.assign(nb, qgt_block_tuning{});
    P.tuning_src.assign(nb, 0);
    const std::string pclass = cache.empty() ? std::string() : plan_class(P.blocks);
    for (int gg = 0; gg < nb; ++gg) {
      BlockDev& bd = P.blocks[gg];
      if (opts && opts->tuning) {
        P.tuning[gg] = opts->tuning[gg];
        P.tuning_src[gg] = 1;
      } else if (!cache.blocks.empty()) {
        const std::string cls = tune_class(bd);
        auto it = cache.blocks.find(plan_block_key(pclass, cls));
        P.tuning_src[gg] = 3;
        if (it == cache.blocks.end()) {
          it = cache.blocks.find(cls);
          P.tuning_src[gg] = 2;
        }
        if (it == cache.blocks.end()) {
          P.tuning_src[gg] = 0;
        } else {
          P.tuning[gg] = it->second;
          if ((P.tuning[gg].gram_tile == 2 && !wide_eligible(bd)) || (P.tuning[gg].gram_tile == 3 && bd.prec != PREC_BF16))
            P.tuning[gg].gram_tile = 0;
        }
      }
      st = resolve_tuning(bd, P.tuning[gg]);
      if (st != QGT_OK) return st;
      bd.chunk = P.tuning[gg].chol_chunk;
    }
    // how the factorisations launch: the caller's choice, else the mode the
    // autotuner measured faster for this set of blocks, else the persistent
    // launch
    const int32_t asked = opts ? opts->cholesky : QGT_CHOL_AUTO;
    int32_t mode = asked == QGT_CHOL_AUTO ? QGT_CHOL_PERSISTENT : asked;
    P.chol_mode_src = asked == QGT_CHOL_AUTO ? 0 : 1;
    if (asked == QGT_CHOL_AUTO && !cache.plans.empty()) {
      auto it = cache.plans.find(pclass);
      if (it != cache.plans.end() && (it->second == QGT_CHOL_HOST_STEPS || it->second == QGT_CHOL_PERSISTENT)) {
        mode = it->second;
        P.chol_mode_src = 2;
      }
    }
    P.chol_host_steps = mode == QGT_CHOL_HOST_STEPS;
  }
  P.status_off = L.take(sizeof(int32_t) * nb);
  P.floor_off = L.take(sizeof(int32_t) * nb);
  P.bscal_off = L.take(sizeof(double2) * nb);
  P.trace_off = L.take(sizeof(double) * nb);
  P.cg_off = L.take(sizeof(CgScal) * nb);
  for (auto& pd : P.probs) {
    pd.dE_off = L.take(16 * pd.n_s);
    pd.mu_off = L.take(16 * pd.n_p);
    pd.F_off = L.take(16 * pd.n_p);
    pd.v_off = L.take(16 * pd.n_p);
    pd.sd_off = L.take(8 * pd.n_p);
    pd.scal_off = L.take(16 * 4);
  }
  for (size_t g = 0; g < P.blocks.size(); ++g) {
    BlockDev& bd = P.blocks[g];
    const ProbDev& pd = P.probs[bd.prob];
    bd.tr_off = P.trace_off + (int64_t)(8 * g);
    bd.cg_off = P.cg_off + (int64_t)(sizeof(CgScal) * g);
    bd.pack_off = L.take((size_t)2 * bd.K_pad * bd.m_pad * prec_bytes(bd.prec));
    bd.mat_off = L.take((size_t)bd.m_pad * bd.m_pad * factor_bytes(bd.fact32 != 0));
    bd.linv_off = L.take((size_t)bd.ntiles * 4096 * factor_bytes(bd.fact32 != 0));
    bd.x_off = L.take((size_t)bd.m_pad * 16);
    bd.r_off = L.take((size_t)bd.m_pad * 16);
    bd.y_off = L.take((size_t)bd.m_pad * 16);
    bd.z_off = L.take((size_t)bd.m_pad * 16);
    bd.p_off = L.take((size_t)bd.m_pad * 16);
    bd.q_off = L.take((size_t)bd.m_pad * 16);
    bd.u_off = L.take((size_t)pd.n_s * 16);
    P.max_mpad = std::max(P.max_mpad, bd.m_pad);
    P.max_nb = std::max(P.max_nb, bd.n_b);
  }

  // Column-pass tiles and row-pass items.
  int64_t min_ns = INT64_MAX;
  for (auto& pd : P.probs) min_ns = std::min(min_ns, pd.n_s);
  for (int gg = 0; gg < nb; ++gg) {
    const BlockDev& bd = P.blocks[gg];
    const ProbDev& pd = P.probs[bd.prob];
    for (int64_t c0 = 0; c0 < bd.n_b; c0 += 64) {
      ColTile t{gg, (int32_t)c0, (int32_t)std::min<int64_t>(64, bd.n_b - c0), 0};
      P.col_all.push_back(t);
      if (bd.form == FORM_S) P.col_s.push_back(t);
    }
    for (int64_t r0 = 0; r0 < pd.n_s; r0 += 16) {
      RowItem it{gg, (int32_t)r0, 0, 0};
      (bd.form == FORM_P ? P.row_p : P.row_s).push_back(it);
    }
    (bd.form == FORM_P ? P.gl_p : P.gl_s).push_back(gg);
    P.gl_pack[bd.form == FORM_P ? 0 : 1][bd.prec].push_back(gg);
  }
  // Row chunks of the column pass: a function of n_s only, so that a problem
  // gives bit-identical results alone or batched with others.
  P.RC = 1;
  for (auto& pd : P.probs) {
    pd.rc = (int32_t)std::max<int64_t>(1, std::min<int64_t>(pd.n_s / 256, 64));
    P.RC = std::max(P.RC, (int)pd.rc);
  }
  (void)min_ns;
  P.colpart_off = L.take((size_t)P.col_all.size() * P.RC * 64 * 48);

  // Pack launch shapes per (form, precision).
  for (int f = 0; f < 2; ++f)
    for (int pr = 0; pr < 3; ++pr) {
      int64_t maxmt = 0, maxgroups = 0;
      for (int gg : P.gl_pack[f][pr]) {
        const BlockDev& bd = P.blocks[gg];
        maxmt = std::max(maxmt, bd.m_pad / 64);
        maxgroups = std::max(maxgroups, bd.K_pad / pack_group(pr));
      }
      if (f == 0) {  // parameter form: 64-column strips, k-groups strided over the y grid
        P.pack_maxmt[f][pr] = maxmt;
        P.pack_ygrid[f][pr] = (int)std::max<int64_t>(1, std::min<int64_t>((maxgroups + 31) / 32, 1024));
      } else {       // sample form: 64 * kPackRowsS rows by 4 k-groups per workgroup
        P.pack_maxmt[f][pr] = (maxmt + kPackRowsS - 1) / kPackRowsS;
        P.pack_ygrid[f][pr] = (int)std::max<int64_t>(1, std::min<int64_t>(maxgroups / 4, 16384));
      }
    }

  // Gram work items: lower-triangle tiles of every block, split along the
  // contraction when there are too few tiles to fill the GPU.  List 3 holds
  // the 256x128 tiles of large BF16 blocks (wide kernel), list 4 the 128x128
  // tiles of BF16 blocks taken two workgroups per CU (duo kernel); neither is
  // split.
  std::vector<SplitItem>& splits = P.split_items;
  int32_t slot = 0;
  auto list_of = [&](int gg) {
    const int tile = P.tuning[gg].gram_tile;
    return tile == 2 ? 3 : (tile == 3 ? 4 : P.blocks[gg].prec);
  };
  for (int li = 0; li < 5; ++li) {
    const int pr = li >= 3 ? PREC_BF16 : li;
    const bool wide = li == 3, unsplit = li >= 3;
    std::vector<int32_t> gl;
    for (int gg = 0; gg < nb; ++gg)
      if (list_of(gg) == li) gl.push_back(gg);
    if (gl.empty()) continue;
    // largest work first
    std::stable_sort(gl.begin(), gl.end(), [&](int a, int b) {
      const BlockDev &A = P.blocks[a], &B = P.blocks[b];
      return (double)A.m_pad * A.m_pad * A.K_pad > (double)B.m_pad * B.m_pad * B.K_pad;
    });
    std::vector<GramItem>& items = P.gram_items[li];
    std::vector<std::vector<GramItem>> per_block;  // each block's items in patch order
    for (int gg : gl) {
      per_block.emplace_back();
      std::vector<GramItem>& bitems = per_block.back();
      const BlockDev& bd = P.blocks[gg];
      const int ks = gram_stage_k(pr);
      const int64_t nst = bd.K_pad / ks;
      // tile rows of RT, tile columns of 128; a tile is kept if it reaches the
      // lower triangle (tj * 128 < (ti + 1) * RT)
      const int RT = wide ? 256 : 128, CPR = RT / 128;
      const int TR = (int)(bd.m_pad / RT), TC = (int)(bd.m_pad / 128);
      const int64_t btiles = (int64_t)CPR * TR * (TR + 1) / 2;
      // split along the contraction so that each block alone yields at least
      // the tuned number of work items (default 256), keeping >= 16 stages
      // per split (a function of the block and its tuning only: batching does
      // not change the summation order)
      const int64_t items = P.tuning[gg].gram_items;
      int64_t split = unsplit ? 1 : std::min<int64_t>((items + btiles - 1) / btiles, std::max<int64_t>(1, nst / 16));
      split = std::max<int64_t>(1, std::min<int64_t>(split, nst));
      // Tiles in patches of gram_patch (default 4) 128-row block rows x 8 block
      // columns: the ~32 tiles one XCD runs at a time then share a few
      // operand panels in its L2 instead of one panel per tile along a single
      // block row.
      std::vector<std::pair<int, int>> order;
      order.reserve((size_t)btiles);
      const int PH = std::max(1, P.tuning[gg].gram_patch / CPR), PW = 8;
      for (int pi = 0; pi * PH < TR; ++pi)
        for (int pj = 0; pj * PW < std::min(TC, (pi * PH + PH) * CPR); ++pj)
          for (int ti = pi * PH; ti < std::min(TR, pi * PH + PH); ++ti)
            for (int tj = pj * PW; tj < std::min((ti + 1) * CPR, pj * PW + PW); ++tj) order.emplace_back(ti, tj);
      for (const auto& tt : order) {
        const int ti = tt.first, tj = tt.second;
        if (split == 1) {
          bitems.push_back(GramItem{gg, ti, tj, 0, (int32_t)nst, -1});
        } else {
          SplitItem si{gg, ti, tj, slot, (int32_t)split, 0};
          for (int64_t sp = 0; sp < split; ++sp) {
            const int32_t s0 = (int32_t)(nst * sp / split), s1 = (int32_t)(nst * (sp + 1) / split);
            bitems.push_back(GramItem{gg, ti, tj, s0, s1, slot++});
          }
          splits.push_back(si);
        }
      }
      P.gram_flops[bd.prec] += bd.form == FORM_P ? 4.0 * (double)P.probs[bd.prob].n_s * bd.n_b * bd.n_b
                                                 : 4.0 * (double)bd.n_b * P.probs[bd.prob].n_s * P.probs[bd.prob].n_s;
    }
    // One list per XCD (workgroup x of the launch runs on XCD x % 8), each
    // holding an eighth of every block's items, contiguous in patch order so
    // that an XCD's concurrent tiles share operand panels in its L2; blocks
    // in order of decreasing work, so that every XCD starts with the longest
    // tiles and ends with the shortest.  Contiguous chunks of equal cost left
    // whole XCDs with only the longest tiles (2.1 per CU on the default
    // workload), whose last round ran a third of the CUs.
    std::vector<std::vector<GramItem>> xl(8);
    for (const auto& bitems : per_block) {
      const int64_t n = (int64_t)bitems.size();
      for (int x = 0; x < 8; ++x)
        for (int64_t i = n * x / 8; i < n * (x + 1) / 8; ++i) xl[x].push_back(bitems[(size_t)i]);
    }
    for (int x = 0; x < 8; ++x) {
      P.gram_xcd[li][x] = (int32_t)items.size();
      P.gram_xcd[li][8 + x] = (int32_t)xl[x].size();
      P.gram_maxlen[li] = std::max<int>(P.gram_maxlen[li], (int)xl[x].size());
      items.insert(items.end(), xl[x].begin(), xl[x].end());
    }
  }
  P.gpart_off = L.take((size_t)std::max<int32_t>(slot, 1) * kGramTile * kGramTile * 16);

  // Blocks sorted by tile count (largest first) for the Cholesky and the
  // triangular solves.
  P.gl_sorted.resize(nb);
  for (int i = 0; i < nb; ++i) P.gl_sorted[i] = i;
  std::stable_sort(P.gl_sorted.begin(), P.gl_sorted.end(),
                   [&](int a, int b) { return P.blocks[a].ntiles > P.blocks[b].ntiles; });
  P.Tmax = P.blocks[P.gl_sorted[0]].ntiles;
  if ((double)P.Tmax * P.Tmax * P.Tmax * nb > 1.5e9) return fail(QGT_ERR_UNSUPPORTED, "too many Cholesky tiles");

  // The persistent Cholesky: every block's tile tasks merged by decreasing
  // bottom level (a topological order of each block's graph, since a task's
  // bottom level exceeds those of all tasks that depend on it), ties in block
  // and column order.
  {
    if (P.Tmax > 32767) return fail(QGT_ERR_UNSUPPORTED, "matrix order above 2^21");
    struct Keyed {
      double bl;
      int64_t nat;
      CholTask t;
    };
    std::vector<Keyed> all;
    std::vector<CholTask> bt;
    std::vector<double> bbl;
    int64_t nat = 0;
    int state = 0;
    for (int gg = 0; gg < nb; ++gg) {
      BlockDev& bd = P.blocks[gg];
      bd.tile_state = state;
      state += bd.ntiles * (bd.ntiles + 1) / 2;
      chol_block_tasks(gg, bd.ntiles, bd.chunk, bt, bbl);
      for (size_t x = 0; x < bt.size(); ++x) all.push_back(Keyed{bbl[x], nat++, bt[x]});
    }
    std::stable_sort(all.begin(), all.end(), [](const Keyed& a, const Keyed& b) {
      return a.bl != b.bl ? a.bl > b.bl : a.nat < b.nat;
    });
    P.chol_tasks.resize(all.size());
    for (size_t x = 0; x < all.size(); ++x) P.chol_tasks[x] = all[x].t;
    P.chol_state_n = state;
    // Self-check: executing the tasks one at a time in ticket order meets
    // every task's wait condition (what guarantees that the device-side waits
    // end), and every tile ends with all its operations done.
    {
      std::vector<int> cnt((size_t)std::max(state, 1), 0);
      auto done_final = [&](const BlockDev& bd, int a, int k) {
        return cnt[(size_t)(bd.tile_state + tri_index(a, k))] == chol_nchunks(k, bd.chunk) + 1;
      };
      for (const CholTask& t : P.chol_tasks) {
        const BlockDev& bd = P.blocks[t.g];
        int& own = cnt[(size_t)(bd.tile_state + tri_index(t.i, t.j))];
        bool ok = own == t.seq;
        if (t.type == CHOL_UPD)
          for (int k = t.k0; k < t.k1; ++k) ok = ok && done_final(bd, t.i, k) && done_final(bd, t.j, k);
        else if (t.type == CHOL_TRSM)
          ok = ok && done_final(bd, t.j, t.j);
        if (!ok) return fail(QGT_ERR_INTERNAL, "Cholesky task order is not topological");
        ++own;
      }
      for (int gg = 0; gg < nb; ++gg) {
        const BlockDev& bd = P.blocks[gg];
        for (int i = 0; i < bd.ntiles; ++i)
          for (int j = 0; j <= i; ++j)
            if (!done_final(bd, i, j)) return fail(QGT_ERR_INTERNAL, "Cholesky task list is incomplete");
      }
    }
    P.chol_state_off = L.take(sizeof(int32_t) * (size_t)std::max(state, 1));
    P.chol_ctl_off = L.take(sizeof(int32_t) * kCholCtl);
    split_chol_queues(P, 8);
  }

  // Triangular-solve tickets: forward in increasing tile order, backward from
  // the last tile of each block, interleaving the blocks step by step.
  P.tile_base.assign(nb, 0);
  int tb = 0;
  for (int gg = 0; gg < nb; ++gg) {
    P.tile_base[gg] = tb;
    tb += P.blocks[gg].ntiles;
  }
  P.total_tiles = tb;
  for (int d = 0; d < P.Tmax; ++d)
    for (int gg : P.gl_sorted) {
      const int T = P.blocks[gg].ntiles;
      if (T > d) {
        P.tmap_fwd.push_back(make_int2(gg, d));
        P.tmap_bwd.push_back(make_int2(gg, T - 1 - d));
      }
    }
  // Right-looking tile Cholesky over pairs of steps (k, k+1), k even (every
  // block has an even number of 64-tiles since m_pad is a multiple of 128).
  // Per step: POTRF of tile (k,k) of every block with ntiles > k and TRSM of
  // the tiles below it.  Per pair: the single-step update of column k+1 from
  // panel k (before step k+1 can be factored), then the trailing update of
  // the pair from both panels at once (K = 128): first columns k+2 and k+3
  // (the lookahead columns, on the critical path), then the rest (j >= k+4).
  for (int k = 0; k < P.Tmax; ++k) {
    int c = 0;
    for (int gg : P.gl_sorted) if (P.blocks[gg].ntiles > k) ++c;
    P.chol_count.push_back(c);
    P.trsm_off.push_back((int32_t)P.trsm_tasks.size());
    for (int gg : P.gl_sorted) {
      const int T = P.blocks[gg].ntiles;
      for (int i = k + 1; i < T; ++i) P.trsm_tasks.push_back(make_int4(gg, i, k, 0));
    }
  }
  for (int k = 0; k < P.Tmax; k += 2) {
    P.upd_off.push_back((int32_t)P.upd_tasks.size());  // column k+1 from panel k
    for (int gg : P.gl_sorted) {
      const int T = P.blocks[gg].ntiles;
      for (int i = k + 1; i < T; ++i) P.upd_tasks.push_back(make_int4(gg, i, k + 1, 0));
    }
    P.upd_col.push_back((int32_t)P.upd_tasks.size());  // columns k+2, k+3 from panels k, k+1
    for (int gg : P.gl_sorted) {
      const int T = P.blocks[gg].ntiles;
      for (int j = k + 2; j < std::min(T, k + 4); ++j)
        for (int i = j; i < T; ++i) P.upd_tasks.push_back(make_int4(gg, i, j, 0));
    }
    P.upd_mid.push_back((int32_t)P.upd_tasks.size());  // the rest, j >= k+4
    for (int gg : P.gl_sorted) {
      const int T = P.blocks[gg].ntiles;
      for (int i = k + 4; i < T; ++i)
        for (int j = k + 4; j <= i; ++j) P.upd_tasks.push_back(make_int4(gg, i, j, 0));
    }
  }
  P.trsm_off.push_back((int32_t)P.trsm_tasks.size());
  P.upd_off.push_back((int32_t)P.upd_tasks.size());
  // Self-check of the triangular-solve tickets: every tile's dependencies must
  // come earlier (this is what guarantees that the device-side waits end).
  {
    std::vector<int> done((size_t)P.total_tiles, 0);
    for (const int2& e : P.tmap_fwd) {
      for (int j = 0; j < e.y; ++j)
        if (!done[P.tile_base[e.x] + j]) return fail(QGT_ERR_INTERNAL, "forward-solve order is not topological");
      done[P.tile_base[e.x] + e.y] = 1;
    }
    std::fill(done.begin(), done.end(), 0);
    for (const int2& e : P.tmap_bwd) {
      for (int j = e.y + 1; j < P.blocks[e.x].ntiles; ++j)
        if (!done[P.tile_base[e.x] + j]) return fail(QGT_ERR_INTERNAL, "backward-solve order is not topological");
      done[P.tile_base[e.x] + e.y] = 1;
    }
  }
  // sync area: [64] forward and [65] backward solve counters; [128 ...] forward
  // flags, then backward flags
  P.sync_ints = 128;
  P.sync_off = L.take((size_t)P.sync_ints * sizeof(int32_t));

  P.ws_bytes = L.bytes;
  return QGT_OK;
}

template <typename T>
int64_t meta_put(std::vector<char>& buf, const std::vector<T>& v) {
  const int64_t off = round_up((int64_t)buf.size(), 256);
  buf.resize(off + std::max<size_t>(v.size(), 1) * sizeof(T), 0);
  if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
  return off;
}

qgt_status upload_plan(qgt_plan_s& P) {
  {
    // one Cholesky ticket queue per XCD (32 compute units each on MI355X)
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0) {
      const int nq = std::max(1, std::min(8, ncu / 32));
      if (nq != P.chol_nq) split_chol_queues(P, nq);
    }
  }
  std::vector<char> buf;
  P.m_probs = meta_put(buf, P.probs);
  P.m_blocks = meta_put(buf, P.blocks);
  P.m_col_all = meta_put(buf, P.col_all);
  P.m_col_s = meta_put(buf, P.col_s);
  P.m_row_p = meta_put(buf, P.row_p);
  P.m_row_s = meta_put(buf, P.row_s);
  P.m_gl_sorted = meta_put(buf, P.gl_sorted);
  P.m_gl_p = meta_put(buf, P.gl_p);
  P.m_gl_s = meta_put(buf, P.gl_s);
  for (int f = 0; f < 2; ++f)
    for (int pr = 0; pr < 3; ++pr) P.m_gl_pack[f][pr] = meta_put(buf, P.gl_pack[f][pr]);
  for (int li = 0; li < 5; ++li) {
    P.m_gram[li] = meta_put(buf, P.gram_items[li]);
    P.m_gram_xcd[li] = meta_put(buf, std::vector<int32_t>(P.gram_xcd[li], P.gram_xcd[li] + 16));
  }
  P.m_split = meta_put(buf, P.split_items);
  P.m_tmap_fwd = meta_put(buf, P.tmap_fwd);
  P.m_tmap_bwd = meta_put(buf, P.tmap_bwd);
  P.m_trsm = meta_put(buf, P.trsm_tasks);
  P.m_upd = meta_put(buf, P.upd_tasks);
  P.m_chol = meta_put(buf, P.chol_qtasks);
  P.m_chol_qoff = meta_put(buf, P.chol_qoff);
  hipError_t e = hipMalloc(&P.dmeta, buf.size());
  if (e != hipSuccess) return fail(QGT_ERR_HIP, std::string("hipMalloc(plan metadata): ") + hipGetErrorString(e));
  e = hipMemcpy(P.dmeta, buf.data(), buf.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(QGT_ERR_HIP, std::string("hipMemcpy(plan metadata): ") + hipGetErrorString(e));
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess) P.device = dev;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
      P.n_cu = ncu;
  }
  const hipError_t se = hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking);
  if (se != hipSuccess ||
      hipEventCreateWithFlags(&P.ev_main, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&P.ev_side, hipEventDisableTiming) != hipSuccess)
    return fail(QGT_ERR_HIP, "stream or event creation failed");
  if (P.timing) {
    for (int pr = 0; pr < 3; ++pr) {
      if (!P.has_gram(pr)) continue;
      P.tpairs[pr].resize(32);
      for (auto& tp : P.tpairs[pr]) {
        if (hipEventCreate(&tp.a) != hipSuccess || hipEventCreate(&tp.b) != hipSuccess)
          return fail(QGT_ERR_HIP, "hipEventCreate failed");
      }
    }
  }
  return QGT_OK;
}

qgt_status check_launch(const char* what) {
  hipError_t e = hipPeekAtLastError();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(QGT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  }
  return QGT_OK;
}

void timing_collect(qgt_plan_s& P, int pr, TimingPair& tp) {
  if (!tp.pending) return;
  float ms = 0.f;
  if (hipEventSynchronize(tp.b) == hipSuccess && hipEventElapsedTime(&ms, tp.a, tp.b) == hipSuccess) {
    P.t_total_ms[pr] += ms;
    P.t_launches[pr] += 1;
  }
  tp.pending = false;
}

void exec_form(qgt_plan_s& P, hipStream_t s) {
  const BlockDev* blocks = P.dev<BlockDev>(P.m_blocks);
  const ProbDev* probs = P.dev<ProbDev>(P.m_probs);
  ProbPtrs* ptrs = reinterpret_cast<ProbPtrs*>(P.ws + P.ptrs_off);
  char* ws = P.ws;
  launch_bind(P.bind, P.nprob, ptrs, s);
  launch_eloc(probs, ptrs, ws, P.nprob, s);
  launch_colpass(P.dt, COL_FORCE, P.dev<ColTile>(P.m_col_all), (int)P.col_all.size(), P.RC, blocks, probs, ptrs, ws,
                 reinterpret_cast<double2*>(ws + P.colpart_off), s);
  launch_block_trace(blocks, probs, ws, reinterpret_cast<double*>(ws + P.trace_off), (int)P.blocks.size(), s);
  for (int f = 0; f < 2; ++f)
    for (int pr = 0; pr < 3; ++pr)
      launch_pack(P.dt, pr, P.dev<int32_t>(P.m_gl_pack[f][pr]), (int)P.gl_pack[f][pr].size(), P.pack_maxmt[f][pr],
                  P.pack_ygrid[f][pr], blocks, probs, ptrs, ws, f == 0 ? FORM_P : FORM_S, s);
  double2* gpart = reinterpret_cast<double2*>(ws + P.gpart_off);
  for (int pr = 0; pr < 3; ++pr) {
    if (!P.has_gram(pr)) continue;
    TimingPair* tp = nullptr;
    if (P.timing) {  // events on the launch stream around this precision's Gram launch
      tp = &P.tpairs[pr][P.tnext[pr]];
      P.tnext[pr] = (P.tnext[pr] + 1) % P.tpairs[pr].size();
      timing_collect(P, pr, *tp);
      (void)hipEventRecord(tp->a, s);
    }
    launch_gram(pr, P.dev<GramItem>(P.m_gram[pr]), P.gram_maxlen[pr], P.dev<int32_t>(P.m_gram_xcd[pr]),
                P.dev<int32_t>(P.m_gram_xcd[pr]) + 8, blocks, ws, gpart, s);
    if (pr == PREC_BF16) {
      launch_gram_wide(P.dev<GramItem>(P.m_gram[3]), P.gram_maxlen[3], P.dev<int32_t>(P.m_gram_xcd[3]),
                       P.dev<int32_t>(P.m_gram_xcd[3]) + 8, blocks, ws, s);
      launch_gram_duo(P.dev<GramItem>(P.m_gram[4]), P.gram_maxlen[4], P.dev<int32_t>(P.m_gram_xcd[4]),
                      P.dev<int32_t>(P.m_gram_xcd[4]) + 8, blocks, ws, s);
    }
    if (tp) {
      (void)hipEventRecord(tp->b, s);
      tp->pending = true;
    }
  }
  launch_gram_splitk_reduce(P.dev<SplitItem>(P.m_split), (int)P.split_items.size(), blocks, ws, gpart, s);
}

void exec_solve(qgt_plan_s& P, hipStream_t s) {
  const BlockDev* blocks = P.dev<BlockDev>(P.m_blocks);
  const ProbDev* probs = P.dev<ProbDev>(P.m_probs);
  ProbPtrs* ptrs = reinterpret_cast<ProbPtrs*>(P.ws + P.ptrs_off);
  char* ws = P.ws;
  const int nb = (int)P.blocks.size();
  int32_t* status = reinterpret_cast<int32_t*>(ws + P.status_off);
  int32_t* floors = reinterpret_cast<int32_t*>(ws + P.floor_off);
  double2* bscal = reinterpret_cast<double2*>(ws + P.bscal_off);
  double2* colpart = reinterpret_cast<double2*>(ws + P.colpart_off);
  const int32_t* gls = P.dev<int32_t>(P.m_gl_sorted);
  launch_bind(P.bind, P.nprob, ptrs, s);
  launch_fill_i32(status, nb, 0, s);
  launch_fill_i32(floors, nb, 0, s);

  if (!P.chol_host_steps) {
    // the Cholesky of every block in one persistent launch over the tile DAG
    int* cstate = reinterpret_cast<int*>(ws + P.chol_state_off);
    int* cctl = reinterpret_cast<int*>(ws + P.chol_ctl_off);
    launch_fill_i32(cstate, P.chol_state_n, 0, s);
    launch_fill_i32(cctl, kCholCtl, 0, s);
    const int nt = (int)P.chol_qtasks.size();
    launch_chol(P.dev<CholTask>(P.m_chol), P.dev<int32_t>(P.m_chol_qoff), P.chol_nq, nt, 2 * P.n_cu, blocks, ws,
                cstate, cctl, status, floors, s);
  } else {
    // Cholesky, right-looking over tile columns in pairs of steps with
    // lookahead: the bulk of a pair's trailing update (columns >= k+4, K = 128)
    // runs on the side stream while the caller's stream updates columns k+2 and
    // k+3 and factors the next pair; the caller's stream waits for the side
    // stream only before it updates columns the side stream has touched.  Event
    // records and waits keep this capturable in a graph.
    auto trsm = [&](int k) {
      launch_tile_gemm(0, P.dev<int4>(P.m_trsm) + P.trsm_off[k], P.trsm_off[k + 1] - P.trsm_off[k], blocks, ws, k, s);
    };
    const int4* upd = P.dev<int4>(P.m_upd);
    launch_potrf(gls, P.chol_count[0], blocks, ws, 0, status, floors, s);
    trsm(0);
    bool side_live = false;
    for (int k = 0, p = 0; k < P.Tmax; k += 2, ++p) {
      // step k+1: its column gets the update from panel k, then is factored
      launch_tile_gemm(1, upd + P.upd_off[p], P.upd_col[p] - P.upd_off[p], blocks, ws, k, s);
      launch_potrf(gls, P.chol_count[k + 1], blocks, ws, k + 1, status, floors, s);
      trsm(k + 1);
      // the side stream's update of an earlier pair covered columns k+2, k+3
      // (only events recorded in this solve are waited for, so that a graph
      // capture never depends on work outside it)
      if (side_live) (void)hipStreamWaitEvent(s, P.ev_side, 0);
      const int n_rest = P.upd_off[p + 1] - P.upd_mid[p], n_next = P.upd_mid[p] - P.upd_col[p];
      if (n_rest + n_next <= 2 * P.n_cu) {
        // a small trailing matrix: one launch on this stream covers columns
        // k+2, k+3 and the rest in about the time of the first two alone, and
        // saves the fork and join of the side stream
        launch_tile_gemm(2, upd + P.upd_col[p], n_next + n_rest, blocks, ws, k, s);
      } else {
        (void)hipEventRecord(P.ev_main, s);
        (void)hipStreamWaitEvent(P.side, P.ev_main, 0);
        launch_tile_gemm(2, upd + P.upd_mid[p], n_rest, blocks, ws, k, P.side);
        (void)hipEventRecord(P.ev_side, P.side);
        side_live = true;
        launch_tile_gemm(2, upd + P.upd_col[p], n_next, blocks, ws, k, s);
      }
      if (k + 2 < P.Tmax) {
        launch_potrf(gls, P.chol_count[k + 2], blocks, ws, k + 2, status, floors, s);
        trsm(k + 2);
      }
    }
    if (side_live) (void)hipStreamWaitEvent(s, P.ev_side, 0);
  }
  int* sync = reinterpret_cast<int*>(ws + P.sync_off);
  CgScal* cg = reinterpret_cast<CgScal*>(ws + P.cg_off);
  auto precond = [&]() {  // z = M^{-1} r with M = L L^H
    launch_fill_i32(sync + 64, 2, 0, s);
    launch_trsv_reset(blocks, ws, nb, P.max_mpad, s);
    const int nt = (int)P.tmap_fwd.size();
    launch_trsv(0, P.dev<int2>(P.m_tmap_fwd), nt, blocks, ws, sync + 64, status, s);
    launch_trsv(1, P.dev<int2>(P.m_tmap_bwd), nt, blocks, ws, sync + 65, status, s);
  };

  // Preconditioned CG in FP64 from x = 0: each iteration applies the shifted
  // operator to the search direction matrix-free from O (row and column passes)
  // and preconditions with the Cholesky factor; a last correction x += M^{-1} r
  // closes the iteration.  max_refine = 0 is the plain solve x = M^{-1} rhs.
  launch_init_solve(blocks, probs, ws, nb, P.max_mpad, s);
  precond();
  launch_cg(CG_START, blocks, ws, cg, P.rtol, P.max_refine, status, nb, s);
  for (int it = 1; it <= P.max_refine; ++it) {
    launch_mudot(P.dev<int32_t>(P.m_gl_p), (int)P.gl_p.size(), blocks, probs, ws, bscal, s);
    launch_rowpass(P.dt, ROW_P_U, P.dev<RowItem>(P.m_row_p), (int)P.row_p.size(), blocks, probs, ptrs, ws, bscal, s);
    launch_colpass(P.dt, COL_APPLY, P.dev<ColTile>(P.m_col_all), (int)P.col_all.size(), P.RC, blocks, probs, ptrs, ws,
                   colpart, s);
    launch_mudot(P.dev<int32_t>(P.m_gl_s), (int)P.gl_s.size(), blocks, probs, ws, bscal, s);
    launch_rowpass(P.dt, ROW_S_APPLY, P.dev<RowItem>(P.m_row_s), (int)P.row_s.size(), blocks, probs, ptrs, ws, bscal,
                   s);
    launch_cg(CG_ALPHA, blocks, ws, cg, P.rtol, P.max_refine, status, nb, s);
    precond();
    if (it < P.max_refine) launch_cg(CG_BETA, blocks, ws, cg, P.rtol, P.max_refine, status, nb, s);
  }
  launch_cg(CG_FINAL, blocks, ws, cg, P.rtol, P.max_refine, status, nb, s);
  launch_scatter_p(blocks, ptrs, ws, nb, P.max_nb, s);
  launch_colpass(P.dt, COL_BACKPROJ, P.dev<ColTile>(P.m_col_s), (int)P.col_s.size(), P.RC, blocks, probs, ptrs, ws,
                 colpart, s);
}

// Cache of single-block FP64 plans for qgt_full_solve.  Each entry holds its
// own mutex: a call enqueues form and solve while holding it, so that calls of
// the same shape (which share the plan's bound pointers, side stream and
// events) do not interleave.
struct FullKey {
  int64_t n_s, n_p;
  double lambda;
  int dt;
  bool operator<(const FullKey& o) const {
    if (n_s != o.n_s) return n_s < o.n_s;
    if (n_p != o.n_p) return n_p < o.n_p;
    if (lambda != o.lambda) return lambda < o.lambda;
    return dt < o.dt;
  }
};
struct FullEntry {
  qgt_plan_s* plan = nullptr;
  std::mutex mu;
};
std::mutex g_full_mu;
std::map<FullKey, FullEntry*> g_full_cache;

// ---------------------------------------------------------------------------
// Device formation of O: workspace layout and launch sequence.
// ---------------------------------------------------------------------------
constexpr int64_t kJacMaxWidth = 65535;
constexpr int64_t kJacMaxSamples = (int64_t)1 << 24;

// Segment table of a row of O and its cut into workgroup tasks.
void jac_add_outer(JacArgs& a, int64_t off, int32_t n_out, int32_t n_in, int32_t g_layer, int32_t v_layer) {
  JacSeg S{};
  S.off = off; S.kind = JAC_OUTER; S.n_out = n_out; S.n_in = n_in; S.g_layer = g_layer; S.v_layer = v_layer;
  S.task0 = a.tasks;
  S.rpi = n_in < 256 ? 256 / n_in : 1;
  // whole 256-lane passes of about kJacTaskElems columns per task
  S.jrows = S.rpi * std::max<int32_t>(1, std::min<int32_t>(kJacTaskElems / (S.rpi * n_in), kJacMaxTaskRows / S.rpi));
  a.seg[a.nseg++] = S;
  a.tasks += (n_out + S.jrows - 1) / S.jrows;
}

void jac_add_copy(JacArgs& a, int64_t off, int32_t n_in, int32_t v_layer, int32_t tail_one) {
  JacSeg S{};
  S.off = off; S.kind = JAC_COPY; S.n_in = n_in; S.v_layer = v_layer; S.tail_one = tail_one;
  S.task0 = a.tasks; S.jrows = 1; S.rpi = 1;
  a.seg[a.nseg++] = S;
  a.tasks += 1;
}

qgt_status jac_launch_rows(JacArgs& a, qgt_dtype o_dtype, hipStream_t stream, const char* what) {
  if ((int64_t)a.tasks * a.n_s > ((int64_t)1 << 31) - 1)
    return fail(QGT_ERR_UNSUPPORTED, "n_s * n_p too large for one launch");
  launch_jac_rows(o_dtype == QGT_C64 ? 0 : 1, a, stream);
  return check_launch(what);
}

struct FfnnLayout {
  int64_t n_p = 0;
  std::vector<int64_t> off;      // block offsets in theta and in a row of O (L + readout + 1 entries)
  std::vector<int64_t> tg, h;    // workspace offsets by layer (index 1..L; -1 when absent)
  size_t bytes = 0;
};

// Validates the network description and lays out theta and the workspace.
qgt_status ffnn_layout(const qgt_ffnn* net, int64_t n_s, FfnnLayout& F) {
  if (!net || !net->widths) return fail(QGT_ERR_INVALID_ARGUMENT, "network or widths is null");
  const int L = net->n_layers;
  if (L < 1 || L > kJacMaxLayers)
    return fail(QGT_ERR_UNSUPPORTED, "n_layers must be in [1, " + std::to_string(kJacMaxLayers) + "]");
  if (net->readout != 0 && net->readout != 1) return fail(QGT_ERR_INVALID_ARGUMENT, "readout must be 0 or 1");
  if (n_s < 1 || n_s > kJacMaxSamples) return fail(QGT_ERR_UNSUPPORTED, "n_s must be in [1, 2^24]");
  for (int l = 0; l <= L; ++l)
    if (net->widths[l] < 1 || net->widths[l] > kJacMaxWidth)
      return fail(QGT_ERR_UNSUPPORTED, "width " + std::to_string(l) + " must be in [1, 65535]");
  F.off.assign(1, 0);
  for (int l = 1; l <= L; ++l) {
    F.off.push_back(F.off.back() + (int64_t)net->widths[l] * net->widths[l - 1] + net->widths[l]);
  }
  if (net->readout) F.off.push_back(F.off.back() + net->widths[L] + 1);
  F.n_p = F.off.back();
  if (F.n_p > ((int64_t)1 << 31) - 1) return fail(QGT_ERR_UNSUPPORTED, "n_p above 2^31");
  Layout lay;
  F.tg.assign(L + 1, -1);
  F.h.assign(L + 1, -1);
  for (int l = 1; l <= L; ++l) {
    const size_t arr = (size_t)n_s * net->widths[l] * 16;
    F.tg[l] = lay.take(arr);
    if (l < L || net->readout) F.h[l] = lay.take(arr);
  }
  F.bytes = lay.bytes;
  return QGT_OK;
}

qgt_status jac_common_checks(const void* theta, const int8_t* x, int64_t ldx, int64_t n_in, qgt_dtype o_dtype,
                             const void* O, int64_t ldo, int64_t n_p, const void* ws, size_t ws_bytes,
                             size_t need) {
  if (!theta || !x || !O) return fail(QGT_ERR_INVALID_ARGUMENT, "theta, x or O is null");
  if (o_dtype != QGT_C64 && o_dtype != QGT_C128) return fail(QGT_ERR_INVALID_ARGUMENT, "unknown O dtype");
  if (ldx < n_in) return fail(QGT_ERR_INVALID_ARGUMENT, "ldx < N");
  if (ldo < n_p) return fail(QGT_ERR_INVALID_ARGUMENT, "ldo < n_p");
  if (need > 0 && !ws) return fail(QGT_ERR_INVALID_ARGUMENT, "workspace is null");
  if (ws_bytes < need)
    return fail(QGT_ERR_WORKSPACE_TOO_SMALL, "workspace needs " + std::to_string(need) + " bytes");
  if (((uintptr_t)ws & 255) != 0) return fail(QGT_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
  return QGT_OK;
}

struct CnnLayout {
  int64_t n_p = 0;
  std::vector<int64_t> off;      // block offsets (L + 1 entries)
  std::vector<int64_t> tg, h;    // workspace offsets by layer (index 1..L; -1 when absent)
  size_t bytes = 0;
};

constexpr int32_t kCnnMaxChannels = 16;
constexpr int64_t kCnnMaxLds = 65536;           // bytes of LDS per sample and layer

qgt_status cnn_layout(const qgt_cnn* net, int64_t n_s, CnnLayout& F) {
  if (!net) return fail(QGT_ERR_INVALID_ARGUMENT, "network is null");
  const int L = net->n_layers, C = net->channels, side = net->side;
  if (L < 1 || L > kJacMaxLayers) return fail(QGT_ERR_UNSUPPORTED, "n_layers must be in [1, 8]");
  if (C < 1 || C > kCnnMaxChannels) return fail(QGT_ERR_UNSUPPORTED, "channels must be in [1, 16]");
  // the kernel-derivative pass holds one sample's g and h of a layer and the
  // neighbour map in LDS: (channels + input channels) x 16 B + 18 B per site
  const int64_t lds = ((int64_t)C + (L > 1 ? C : 1)) * side * side * 16 + (int64_t)18 * side * side;
  if (side < 2 || lds > kCnnMaxLds)
    return fail(QGT_ERR_UNSUPPORTED, "side must be >= 2 with (2 channels x 16 + 18) x side^2 <= 65536 bytes");
  if (n_s < 1 || n_s > kJacMaxSamples) return fail(QGT_ERR_UNSUPPORTED, "n_s must be in [1, 2^24]");
  const int64_t S = (int64_t)side * side;
  F.off.assign(1, 0);
  for (int l = 1; l <= L; ++l) {
    const int64_t cin = l == 1 ? 1 : C;
    F.off.push_back(F.off.back() + C * cin * 9 + C);
  }
  F.n_p = F.off.back();
  Layout lay;
  F.tg.assign(L + 1, -1);
  F.h.assign(L + 1, -1);
  for (int l = 1; l <= L; ++l) {
    const size_t arr = (size_t)n_s * C * S * 16;
    F.tg[l] = lay.take(arr);
    if (l < L) F.h[l] = lay.take(arr);
  }
  F.bytes = lay.bytes;
  return QGT_OK;
}

// ---------------------------------------------------------------------------
// Workspace of qgt_block_form_static, for callers that cannot allocate device
// memory: one array per device, resident from the library's first use on that
// device until the process ends.  Host code never passes `scratch` itself to a
// kernel (in host code the name is only a stand-in for the symbol); it uses
// the device address obtained once per device with hipGetSymbolAddress.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = QGT_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (set-up on the first
// call on that device).
qgt_status static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(QGT_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(QGT_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(QGT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return QGT_OK;
}


// ---------------------------------------------------------------------------
// Autotuner support: synthetic inputs for the trials (a counter-based hash:
// splitmix64 of the element index and a seed, mapped to [-1, 1)).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double tune_uniform(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void k_tune_fill(void* p, int64_t n, int c128, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double re = tune_uniform(seed ^ (2 * (uint64_t)i)), im = tune_uniform(seed ^ (2 * (uint64_t)i + 1));
  if (c128) reinterpret_cast<double2*>(p)[i] = make_double2(re, im);
  else reinterpret_cast<float2*>(p)[i] = make_float2((float)re, (float)im);
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) {
    if (p) (void)hipFree(p);
    p = nullptr;
    return hipMalloc(&p, std::max<size_t>(n, 256));
  }
};

// A candidate replaces the best so far only when faster by more than this.
constexpr double kTuneMargin = 0.01;

// The autotuner's progress on stderr, one line per decision, when the
// environment variable QGT_TUNE_LOG is set (non-empty): tuning a set of many
// large blocks takes minutes, and the lines show where it is.
void tune_log(const char* fmt, ...) {
  const char* on = std::getenv("QGT_TUNE_LOG");
  if (!on || !*on) return;
  va_list ap;
  va_start(ap, fmt);
  std::fputs("qgt_autotune: ", stderr);
  std::vfprintf(stderr, fmt, ap);
  std::fputc('\n', stderr);
  va_end(ap);
  std::fflush(stderr);
}

// Milliseconds of fn on the null stream: the fastest of `reps` timed runs
// after one untimed run, the least noisy estimate of what a setting can do
// (clock and power vary between runs).
template <typename F>
qgt_status tune_time(F fn, int reps, double* ms) {
  std::vector<hipEvent_t> ev((size_t)reps + 1, nullptr);
  qgt_status st = QGT_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) st = fail(QGT_ERR_HIP, "hipEventCreate failed");
  if (st == QGT_OK) st = fn();
  if (st == QGT_OK && hipDeviceSynchronize() != hipSuccess) st = fail(QGT_ERR_HIP, "trial failed");
  if (st == QGT_OK) {
    (void)hipEventRecord(ev[0], nullptr);
    for (int r = 0; r < reps && st == QGT_OK; ++r) {
      st = fn();
      (void)hipEventRecord(ev[(size_t)r + 1], nullptr);
    }
    if (st == QGT_OK && hipEventSynchronize(ev[(size_t)reps]) != hipSuccess) st = fail(QGT_ERR_HIP, "trial failed");
    double best = 1e30;
    for (int r = 0; r < reps && st == QGT_OK; ++r) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[(size_t)r], ev[(size_t)r + 1]) != hipSuccess)
        st = fail(QGT_ERR_HIP, "trial timing failed");
      best = std::min(best, (double)t);
    }
    *ms = best;
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  return st;
}

// Writes the cache: the entries of `cache`, one per line, atomically.
bool write_tune_cache(const char* path, const TuneCache& cache,
                      const std::map<std::string, std::pair<double, double>>& times) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\n \"format\": \"qgt-tune-1\",\n \"entries\": {\n");
  const size_t n = cache.blocks.size() + cache.plans.size();
  size_t k = 0;
  for (const auto& kv : cache.blocks) {
    const qgt_block_tuning& t = kv.second;
    std::fprintf(f, "  \"%s\": {\"gram_tile\": %d, \"gram_items\": %d, \"chol_chunk\": %d, \"gram_patch\": %d",
                 kv.first.c_str(), t.gram_tile, t.gram_items, t.chol_chunk, t.gram_patch);
    auto it = times.find(kv.first);
    if (it != times.end()) std::fprintf(f, ", \"form_ms\": %.4f, \"step_ms\": %.4f", it->second.first, it->second.second);
    std::fprintf(f, "}%s\n", ++k < n ? "," : "");
  }
  for (const auto& kv : cache.plans) {
    std::fprintf(f, "  \"%s\": {\"cholesky\": %d", kv.first.c_str(), kv.second);
    auto it = times.find(kv.first);
    if (it != times.end())
      std::fprintf(f, ", \"persistent_ms\": %.4f, \"host_steps_ms\": %.4f", it->second.first, it->second.second);
    std::fprintf(f, "}%s\n", ++k < n ? "," : "");
  }
  std::fprintf(f, " }\n}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace


namespace qgt {
// Error reporting for the entry points defined in other translation units.
qgt_status report_error(qgt_status s, const char* msg) { return fail(s, msg); }
qgt_status report_launch(const char* what) { return check_launch(what); }
}  // namespace qgt

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

qgt_status qgt_block_workspace_query(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype,
                                     qgt_precision gram, int32_t max_refine, const qgt_plan_options* opts,
                                     size_t* workspace_bytes) {
  try {
    if (!workspace_bytes) return fail(QGT_ERR_INVALID_ARGUMENT, "workspace_bytes is null");
    qgt_plan_s P;
    qgt_status st = build_plan(probs, n_probs, o_dtype, gram, max_refine, opts, P);
    if (st != QGT_OK) return st;
    *workspace_bytes = P.ws_bytes;
    return QGT_OK;
  } catch (const std::bad_alloc&) {
    return fail(QGT_ERR_INVALID_ARGUMENT, "out of host memory while planning");
  } catch (...) {
    return fail(QGT_ERR_INVALID_ARGUMENT, "unexpected error while planning");
  }
}

qgt_status qgt_block_tuning_query(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype,
                                  qgt_precision gram, const qgt_plan_options* opts, int32_t g,
                                  qgt_block_tuning* tuning, int32_t* source) {
  try {
    if (!tuning || !source) return fail(QGT_ERR_INVALID_ARGUMENT, "null output");
    qgt_plan_s P;
    qgt_status st = build_plan(probs, n_probs, o_dtype, gram, 0, opts, P);
    if (st != QGT_OK) return st;
    if (g < 0 || g >= (int32_t)P.blocks.size()) return fail(QGT_ERR_INVALID_ARGUMENT, "bad block index");
    *tuning = P.tuning[g];
    *source = P.tuning_src[g];
    return QGT_OK;
  } catch (...) {
    return fail(QGT_ERR_INVALID_ARGUMENT, "unexpected error while planning");
  }
}

qgt_status qgt_cholesky_query(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype, qgt_precision gram,
                              const qgt_plan_options* opts, int32_t* mode, int32_t* source) {
  try {
    if (!mode || !source) return fail(QGT_ERR_INVALID_ARGUMENT, "null output");
    qgt_plan_s P;
    qgt_status st = build_plan(probs, n_probs, o_dtype, gram, 0, opts, P);
    if (st != QGT_OK) return st;
    *mode = P.chol_host_steps ? QGT_CHOL_HOST_STEPS : QGT_CHOL_PERSISTENT;
    *source = P.chol_mode_src;
    return QGT_OK;
  } catch (...) {
    return fail(QGT_ERR_INVALID_ARGUMENT, "unexpected error while planning");
  }
}

qgt_status qgt_autotune(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype, qgt_precision gram,
                        const char* cache_path, int32_t reps, int32_t* n_classes) {
  try {
    if (!cache_path || !n_classes) return fail(QGT_ERR_INVALID_ARGUMENT, "null cache path or output");
    if (reps < 1 || reps > 1000) return fail(QGT_ERR_INVALID_ARGUMENT, "reps must be in [1, 1000]");
    *n_classes = 0;
    qgt_plan_s P0;
    qgt_status st = build_plan(probs, n_probs, o_dtype, gram, 0, nullptr, P0, false);
    if (st != QGT_OK) return st;
    bool ok = true;
    TuneCache cache = read_tune_cache(cache_path, &ok);
    if (!ok) {
      FILE* f = std::fopen(cache_path, "r");
      if (f) {
        std::fclose(f);
        return fail(QGT_ERR_INTERNAL, std::string("cannot read tuning cache ") + cache_path);
      }
    }
    const int nb = (int)P0.blocks.size();
    // shape classes, largest Gram work first; the blocks of each
    std::vector<std::string> keys;
    std::map<std::string, std::vector<int>> members;
    std::map<std::string, double> work;
    for (int g = 0; g < nb; ++g) {
      const BlockDev& bd = P0.blocks[g];
      const std::string key = tune_class(bd);
      if (!members.count(key)) keys.push_back(key);
      members[key].push_back(g);
      work[key] += (double)bd.m_pad * bd.m_pad * bd.K_pad;
    }
    std::stable_sort(keys.begin(), keys.end(), [&](const std::string& a, const std::string& b) {
      return work[a] > work[b];
    });
    // classes with under 2% of the set's Gram work keep the defaults: their
    // choices do not show in the set's time (and would cost a trial each)
    {
      double total = 0.0;
      for (const std::string& k : keys) total += work[k];
      while (keys.size() > 1 && work[keys.back()] < 0.02 * total) keys.pop_back();
    }
    // synthetic inputs of every problem: the whole set is timed, so that each
    // class is tuned inside the launches it shares with the others
    const size_t esz = o_dtype == QGT_C64 ? 8 : 16;
    std::vector<DevBuf> O(n_probs), E(n_probs), D(n_probs);
    std::vector<const void*> Op(n_probs), Ep(n_probs);
    std::vector<void*> Dp(n_probs);
    std::vector<int64_t> ld(n_probs);
    for (int p = 0; p < n_probs; ++p) {
      const int64_t n_s = P0.probs[p].n_s, n_p = P0.probs[p].n_p;
      if (O[p].alloc((size_t)n_s * n_p * esz) != hipSuccess || E[p].alloc((size_t)n_s * 16) != hipSuccess ||
          D[p].alloc((size_t)n_p * 16) != hipSuccess)
        return fail(QGT_ERR_HIP, "hipMalloc of the trial inputs failed");
      hipLaunchKernelGGL(k_tune_fill, dim3((unsigned)((n_s * n_p + 255) / 256)), dim3(256), 0, nullptr, O[p].p,
                         n_s * n_p, o_dtype == QGT_C128 ? 1 : 0, (uint64_t)0x5EEDull + p);
      hipLaunchKernelGGL(k_tune_fill, dim3((unsigned)((n_s + 255) / 256)), dim3(256), 0, nullptr, E[p].p, n_s, 1,
                         (uint64_t)0xE10Cull + p);
      Op[p] = O[p].p;
      Ep[p] = E[p].p;
      Dp[p] = D[p].p;
      ld[p] = n_p;
    }
    if ((st = check_launch("qgt_autotune fill")) != QGT_OK) return st;
    std::vector<int32_t> forms(nb);
    for (int g = 0; g < nb; ++g) forms[g] = P0.blocks[g].form == FORM_P ? QGT_FORM_PARAM : QGT_FORM_SAMPLE;
    std::vector<qgt_block_tuning> cur(nb, qgt_block_tuning{0, 0, 0, 0});
    DevBuf W;
    // time the whole set's form step (with_solve: form + solve) under `cur`,
    // with the factorisations launched as `mode` (the chunk only shapes the
    // persistent launch)
    auto trial = [&](bool with_solve, double* ms, int32_t mode = QGT_CHOL_PERSISTENT) -> qgt_status {
      qgt_plan_options o{};
      o.forms = forms.data();
      o.tuning = cur.data();
      o.cholesky = mode;
      qgt_plan plan = nullptr;
      size_t wsb = 0;
      qgt_status s2 = qgt_block_plan_ex(probs, n_probs, o_dtype, gram, 0, 0.0, &o, &plan, &wsb);
      if (s2 != QGT_OK) return s2;
      if (W.alloc(wsb) != hipSuccess) {
        qgt_plan_destroy(plan);
        return fail(QGT_ERR_HIP, "hipMalloc of the trial workspace failed");
      }
      s2 = tune_time(
          [&]() {
            qgt_status r = qgt_block_form(plan, Op.data(), ld.data(), Ep.data(), W.p, wsb, nullptr);
            if (r == QGT_OK && with_solve) r = qgt_block_solve(plan, Dp.data(), nullptr);
            return r;
          },
          reps, ms);
      qgt_plan_destroy(plan);
      return s2;
    };
    auto set_class = [&](const std::string& key, const qgt_block_tuning& t) {
      for (int g : members[key]) cur[g] = t;
    };
    // coordinate descent, one class at a time (largest first): the Gram's
    // tile shape, split and patch order on the form step, then the Cholesky
    // chunk on form + solve; the default comes first and a later candidate
    // replaces the best so far only if it is faster by more than kTuneMargin
    double form_ms = 0.0, step_ms = 0.0;
    for (const std::string& key : keys) {
      const BlockDev& bd = P0.blocks[members[key][0]];
      std::vector<qgt_block_tuning> grams;
      for (int tile = 1; tile <= 3; ++tile)
        for (int items : {256, 512, 1024})
          for (int patch : {4, 2, 8, 16}) {
            if (tile == 2 && !wide_eligible(bd)) continue;
            if (tile == 3 && bd.prec != PREC_BF16) continue;
            if (tile >= 2 && items != 256) continue;  // the wide and duo kernels are never split
            grams.push_back(qgt_block_tuning{tile, items, 0, patch});
          }
      if (wide_eligible(bd))  // the default (wide tiles, patch 4) first
        std::rotate(grams.begin(), std::find_if(grams.begin(), grams.end(),
                                                [](const qgt_block_tuning& c) { return c.gram_tile == 2; }),
                    grams.end());
      qgt_block_tuning best = grams[0];
      double best_ms = 1e30;
      for (const qgt_block_tuning& c : grams) {
        set_class(key, c);
        double ms = 0.0;
        if ((st = trial(false, &ms)) != QGT_OK) return st;
        if (ms < best_ms * (1.0 - kTuneMargin)) {
          best_ms = ms;
          best = c;
        }
      }
      set_class(key, best);
      form_ms = best_ms;
      tune_log("%s: Gram tile %d, items %d, patch %d: form step %.3f ms", key.c_str(), best.gram_tile,
               best.gram_items, best.gram_patch, best_ms);
    }
    // one tile kind for every BF16 class at once: the classes share their
    // launch, so a kind that only pays when all blocks take it is missed by
    // the one-class moves above
    for (int tile = 1; tile <= 3; ++tile) {
      std::vector<qgt_block_tuning> trial_cur = cur, saved = cur;
      int changed = 0;
      for (const std::string& key : keys) {
        const BlockDev& bd = P0.blocks[members[key][0]];
        if (bd.prec != PREC_BF16 || (tile == 2 && !wide_eligible(bd))) continue;
        qgt_block_tuning c = cur[members[key][0]];
        if (c.gram_tile == tile) continue;
        c.gram_tile = tile;
        if (tile >= 2) c.gram_items = 256;
        for (int g : members[key]) trial_cur[g] = c;
        ++changed;
      }
      if (changed < 2) continue;
      cur = trial_cur;
      double ms = 0.0;
      if ((st = trial(false, &ms)) != QGT_OK) return st;
      const bool taken = ms < form_ms * (1.0 - kTuneMargin);
      tune_log("Gram tile %d for every BF16 class: form step %.3f ms against %.3f ms (%s)", tile, ms, form_ms,
               taken ? "taken" : "not taken");
      if (taken) form_ms = ms;
      else cur = saved;
    }
    for (const std::string& key : keys) {
      qgt_block_tuning best = cur[members[key][0]];
      double best_ms = 1e30;
      for (int chunk : {4, 1, 2, 3, 6, 8, 12}) {
        qgt_block_tuning c = best;
        c.chol_chunk = chunk;
        set_class(key, c);
        double ms = 0.0;
        if ((st = trial(true, &ms)) != QGT_OK) return st;
        if (ms < best_ms * (1.0 - kTuneMargin)) {
          best_ms = ms;
          best.chol_chunk = chunk;
        }
      }
      set_class(key, best);
      step_ms = best_ms;
      tune_log("%s: Cholesky chunk %d: form + solve %.3f ms", key.c_str(), best.chol_chunk, best_ms);
    }
    // each class's choice for this set of blocks, and as the class's own
    // entry (for sets never tuned)
    std::map<std::string, std::pair<double, double>> times;
    const std::string pk = plan_class(P0.blocks);
    for (const std::string& key : keys) {
      qgt_block_tuning t = cur[members[key][0]];
      const BlockDev& bd = P0.blocks[members[key][0]];
      (void)resolve_tuning(bd, t);
      cache.blocks[key] = t;
      cache.blocks[plan_block_key(pk, key)] = t;
      times[key] = std::make_pair(form_ms, step_ms);
      ++*n_classes;
    }
    // the launch mode of the factorisations for this set of blocks: the
    // host-sequenced steps only where they are faster by more than the margin
    {
      double t_p = 0.0, t_h = 0.0;
      if ((st = trial(true, &t_p, QGT_CHOL_PERSISTENT)) != QGT_OK) return st;
      if ((st = trial(true, &t_h, QGT_CHOL_HOST_STEPS)) != QGT_OK) return st;
      cache.plans[pk] = t_h < t_p * (1.0 - kTuneMargin) ? QGT_CHOL_HOST_STEPS : QGT_CHOL_PERSISTENT;
      times[pk] = std::make_pair(t_p, t_h);
      tune_log("%s: Cholesky persistent %.3f ms, host steps %.3f ms", pk.c_str(), t_p, t_h);
    }
    if (!write_tune_cache(cache_path, cache, times))
      return fail(QGT_ERR_INTERNAL, std::string("cannot write tuning cache ") + cache_path);
    return QGT_OK;
  } catch (...) {
    return fail(QGT_ERR_HIP, "unexpected error in qgt_autotune");
  }
}

qgt_status qgt_block_plan_ex(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype, qgt_precision gram,
                             int32_t max_refine, double refine_rtol, const qgt_plan_options* opts, qgt_plan* out,
                             size_t* workspace_bytes) {
  try {
    if (!out || !workspace_bytes) return fail(QGT_ERR_INVALID_ARGUMENT, "out or workspace_bytes is null");
    *out = nullptr;
    if (!(refine_rtol >= 0.0) || refine_rtol == INFINITY)
      return fail(QGT_ERR_INVALID_ARGUMENT, "refine_rtol must be finite and >= 0");
    qgt_plan_s* P = new qgt_plan_s();
    P->rtol = refine_rtol;
    qgt_status st = build_plan(probs, n_probs, o_dtype, gram, max_refine, opts, *P);
    if (st == QGT_OK) st = upload_plan(*P);
    if (st != QGT_OK) {
      delete P;
      return st;
    }
    *out = P;
    *workspace_bytes = P->ws_bytes;
    return QGT_OK;
  } catch (const std::bad_alloc&) {
    return fail(QGT_ERR_INVALID_ARGUMENT, "out of host memory while planning");
  } catch (...) {
    return fail(QGT_ERR_INVALID_ARGUMENT, "unexpected error while planning");
  }
}

qgt_status qgt_block_plan(const qgt_problem* probs, int32_t n_probs, qgt_dtype o_dtype, qgt_precision gram,
                          int32_t max_refine, double refine_rtol, qgt_plan* out, size_t* workspace_bytes) {
  return qgt_block_plan_ex(probs, n_probs, o_dtype, gram, max_refine, refine_rtol, nullptr, out, workspace_bytes);
}

qgt_status qgt_block_form(qgt_plan plan, const void* const* O, const int64_t* ldo, const void* const* e_loc,
                          void* workspace, size_t workspace_bytes, hipStream_t stream) {
  try {
    if (!plan) return fail(QGT_ERR_INVALID_ARGUMENT, "plan is null");
    if (!O || !ldo || !e_loc || !workspace) return fail(QGT_ERR_INVALID_ARGUMENT, "null pointer argument");
    if (workspace_bytes < plan->ws_bytes)
      return fail(QGT_ERR_WORKSPACE_TOO_SMALL, "workspace needs " + std::to_string(plan->ws_bytes) + " bytes");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(QGT_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
    for (int p = 0; p < plan->nprob; ++p) {
      if (!O[p] || !e_loc[p]) return fail(QGT_ERR_INVALID_ARGUMENT, "null O or e_loc for problem " + std::to_string(p));
      if (ldo[p] < plan->probs[p].n_p)
        return fail(QGT_ERR_INVALID_ARGUMENT, "ldo < n_p for problem " + std::to_string(p));
      if (reinterpret_cast<uintptr_t>(O[p]) % 16 != 0 || reinterpret_cast<uintptr_t>(e_loc[p]) % 16 != 0)
        return fail(QGT_ERR_INVALID_ARGUMENT, "O and e_loc must be 16-byte aligned");
      plan->bind.p[p].O = O[p];
      plan->bind.p[p].ldo = ldo[p];
      plan->bind.p[p].e_loc = reinterpret_cast<const double2*>(e_loc[p]);
      plan->bind.p[p].delta = nullptr;
    }
    plan->ws = reinterpret_cast<char*>(workspace);
    exec_form(*plan, stream);
    qgt_status st = check_launch("qgt_block_form");
    if (st == QGT_OK) plan->formed = true;
    return st;
  } catch (...) {
    return fail(QGT_ERR_HIP, "unexpected error in qgt_block_form");
  }
}

qgt_status qgt_block_form_static(qgt_plan plan, const void* const* O, const int64_t* ldo, const void* const* e_loc,
                                 hipStream_t stream) {
  try {
    if (!plan) return fail(QGT_ERR_INVALID_ARGUMENT, "plan is null");
    if (plan->ws_bytes > kStaticScratchBytes)
      return fail(QGT_ERR_WORKSPACE_TOO_SMALL,
                  "the plan needs a workspace of " + std::to_string(plan->ws_bytes) +
                      " bytes; the static workspace of qgt_block_form_static holds " +
                      std::to_string(kStaticScratchBytes) + " bytes (use qgt_block_form with a caller workspace)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
      return fail(QGT_ERR_INVALID_ARGUMENT, "the current device is not the device the plan was made on");
    void* ws = nullptr;
    const qgt_status st = static_scratch(&ws);
    if (st != QGT_OK) return st;
    return qgt_block_form(plan, O, ldo, e_loc, ws, kStaticScratchBytes, stream);
  } catch (...) {
    return fail(QGT_ERR_HIP, "unexpected error in qgt_block_form_static");
  }
}

qgt_status qgt_block_solve(qgt_plan plan, void* const* delta, hipStream_t stream) {
  try {
    if (!plan) return fail(QGT_ERR_INVALID_ARGUMENT, "plan is null");
    if (!plan->formed) return fail(QGT_ERR_INVALID_ARGUMENT, "qgt_block_form has not been called on this plan");
    if (!delta) return fail(QGT_ERR_INVALID_ARGUMENT, "delta is null");
    for (int p = 0; p < plan->nprob; ++p) {
      if (!delta[p]) return fail(QGT_ERR_INVALID_ARGUMENT, "null delta for problem " + std::to_string(p));
      if (reinterpret_cast<uintptr_t>(delta[p]) % 16 != 0)
        return fail(QGT_ERR_INVALID_ARGUMENT, "delta must be 16-byte aligned");
      plan->bind.p[p].delta = reinterpret_cast<double2*>(delta[p]);
    }
    exec_solve(*plan, stream);
    return check_launch("qgt_block_solve");
  } catch (...) {
    return fail(QGT_ERR_HIP, "unexpected error in qgt_block_solve");
  }
}

size_t qgt_full_workspace_bytes(const qgt_problem* p, qgt_dtype o_dtype) {
  if (!p || p->n_blocks < 1 || !p->block_sizes) return 0;
  int64_t np = 0;
  for (int b = 0; b < p->n_blocks; ++b) np += p->block_sizes[b];
  qgt_problem q = *p;
  q.n_blocks = 1;
  q.block_sizes = &np;
  size_t ws = 0;
  if (qgt_block_workspace_query(&q, 1, o_dtype, QGT_GRAM_FP64, 0, nullptr, &ws) != QGT_OK) return 0;
  return ws;
}

qgt_status qgt_full_solve(const qgt_problem* p, qgt_dtype o_dtype, const void* O, int64_t ldo, const void* e_loc,
                          void* delta, void* workspace, size_t ws_bytes, hipStream_t stream) {
  try {
    if (!p || p->n_blocks < 1 || !p->block_sizes) return fail(QGT_ERR_INVALID_ARGUMENT, "invalid problem");
    int64_t np = 0;
    for (int b = 0; b < p->n_blocks; ++b) {
      if (p->block_sizes[b] < 1) return fail(QGT_ERR_INVALID_ARGUMENT, "block size must be positive");
      np += p->block_sizes[b];
    }
    qgt_problem q = *p;
    q.n_blocks = 1;
    q.block_sizes = &np;
    FullKey key{q.n_samples, np, q.lambda, (int)o_dtype};
    FullEntry* entry = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_full_mu);
      auto it = g_full_cache.find(key);
      if (it != g_full_cache.end()) entry = it->second;
    }
    if (!entry) {
      qgt_plan_s* plan = nullptr;
      size_t wsb = 0;
      qgt_status st = qgt_block_plan(&q, 1, o_dtype, QGT_GRAM_FP64, 0, 0.0, &plan, &wsb);
      if (st != QGT_OK) return st;
      std::lock_guard<std::mutex> lk(g_full_mu);
      auto it = g_full_cache.find(key);
      if (it != g_full_cache.end()) {
        delete plan;
        entry = it->second;
      } else {
        entry = new FullEntry();
        entry->plan = plan;
        g_full_cache[key] = entry;
      }
    }
    const void* Op[1] = {O};
    const int64_t ld[1] = {ldo};
    const void* ep[1] = {e_loc};
    void* dp[1] = {delta};
    std::lock_guard<std::mutex> lk(entry->mu);
    qgt_status st = qgt_block_form(entry->plan, Op, ld, ep, workspace, ws_bytes, stream);
    if (st != QGT_OK) return st;
    return qgt_block_solve(entry->plan, dp, stream);
  } catch (...) {
    return fail(QGT_ERR_HIP, "unexpected error in qgt_full_solve");
  }
}

void qgt_full_release(void) {
  std::lock_guard<std::mutex> lk(g_full_mu);
  if (!g_full_cache.empty()) (void)hipDeviceSynchronize();
  for (auto& kv : g_full_cache) {
    {
      std::lock_guard<std::mutex> ek(kv.second->mu);
      delete kv.second->plan;
    }
    delete kv.second;
  }
  g_full_cache.clear();
}

// Scratch layout of qgt_block_inverse_diagnostics: X (largest block, m x m
// complex128), the per-row partial sums and the reference's row norms.
struct DiagLayout {
  int64_t x = 0, part = 0, part2 = 0;
  size_t bytes = 0;
  int64_t ldx = 0;
};
static qgt_status diag_layout(const qgt_plan_s& P, int32_t problem, DiagLayout& D, std::vector<int>& gl,
                              std::vector<int64_t>& ms) {
  if (problem < 0 || problem >= P.nprob) return fail(QGT_ERR_INVALID_ARGUMENT, "bad problem index");
  const ProbDev& pd = P.probs[problem];
  int64_t mmax = 1, rows = 0;
  for (int g = pd.first_block; g < pd.first_block + pd.n_blocks; ++g) {
    const BlockDev& b = P.blocks[g];
    if (b.form != FORM_P)
      return fail(QGT_ERR_UNSUPPORTED, "the inverse diagnostics need every block in parameter form");
    if (b.m > 2048) return fail(QGT_ERR_UNSUPPORTED, "the inverse diagnostics take blocks of order <= 2048");
    gl.push_back(g);
    ms.push_back(b.m);
    mmax = std::max(mmax, b.m);
    rows += b.m;
  }
  Layout L;
  D.ldx = mmax;
  D.x = L.take((size_t)mmax * mmax * 16);
  D.part = L.take((size_t)rows * 5 * 8);
  D.part2 = L.take((size_t)pd.n_p * 8);
  D.bytes = L.bytes;
  return QGT_OK;
}

size_t qgt_block_inverse_scratch_bytes(qgt_plan plan, int32_t problem) {
  if (!plan) return 0;
  DiagLayout D;
  std::vector<int> gl;
  std::vector<int64_t> ms;
  return diag_layout(*plan, problem, D, gl, ms) == QGT_OK ? D.bytes : 0;
}

qgt_status qgt_block_inverse_diagnostics(qgt_plan plan, int32_t problem, const void* B, int64_t ldb, void* scratch,
                                         size_t scratch_bytes, double* sums, hipStream_t stream) {
  try {
    if (!plan || !B || !scratch || !sums) return fail(QGT_ERR_INVALID_ARGUMENT, "null argument");
    if (!plan->formed || !plan->ws) return fail(QGT_ERR_INVALID_ARGUMENT, "the plan has no formed and solved workspace");
    DiagLayout D;
    std::vector<int> gl;
    std::vector<int64_t> ms;
    qgt_status st = diag_layout(*plan, problem, D, gl, ms);
    if (st != QGT_OK) return st;
    const int64_t n_p = plan->probs[problem].n_p;
    if (ldb < n_p) return fail(QGT_ERR_INVALID_ARGUMENT, "ldb < n_p");
    if (scratch_bytes < D.bytes)
      return fail(QGT_ERR_WORKSPACE_TOO_SMALL, "scratch needs " + std::to_string(D.bytes) + " bytes");
    if (reinterpret_cast<uintptr_t>(scratch) % 256 != 0 || reinterpret_cast<uintptr_t>(B) % 16 != 0)
      return fail(QGT_ERR_INVALID_ARGUMENT, "scratch must be 256-byte and B 16-byte aligned");
    char* sc = reinterpret_cast<char*>(scratch);
    launch_block_inverse_sums(plan->dev<BlockDev>(plan->m_blocks), gl, ms, plan->ws,
                              reinterpret_cast<double2*>(sc + D.x), D.ldx, reinterpret_cast<const double2*>(B), ldb,
                              n_p, reinterpret_cast<double*>(sc + D.part), reinterpret_cast<double*>(sc + D.part2), sums,
                              stream);
    return check_launch("qgt_block_inverse_diagnostics");
  } catch (...) {
    return fail(QGT_ERR_HIP, "unexpected error in qgt_block_inverse_diagnostics");
  }
}

qgt_status qgt_plan_status(qgt_plan plan, int32_t* per_block_status) {
  if (!plan || !per_block_status) return fail(QGT_ERR_INVALID_ARGUMENT, "null argument");
  if (!plan->ws) return fail(QGT_ERR_INVALID_ARGUMENT, "no workspace bound");
  const size_t n = plan->blocks.size();
  hipError_t e = hipMemcpy(per_block_status, plan->ws + plan->status_off, n * sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(QGT_ERR_HIP, std::string("hipMemcpy(status): ") + hipGetErrorString(e));
  int32_t worst = 0;
  for (size_t i = 0; i < n; ++i) worst = std::max(worst, per_block_status[i]);
  return (qgt_status)worst;
}

int32_t qgt_plan_num_blocks(qgt_plan plan) { return plan ? (int32_t)plan->blocks.size() : 0; }

qgt_status qgt_plan_block_info(qgt_plan plan, int32_t g, int32_t* problem, int64_t* offset, int64_t* size,
                               int32_t* form, int32_t* precision) {
  if (!plan || g < 0 || g >= (int32_t)plan->blocks.size()) return fail(QGT_ERR_INVALID_ARGUMENT, "bad block index");
  const BlockDev& b = plan->blocks[g];
  if (problem) *problem = b.prob;
  if (offset) *offset = b.col_off;
  if (size) *size = b.n_b;
  if (form) *form = b.form == FORM_P ? QGT_FORM_PARAM : QGT_FORM_SAMPLE;
  if (precision) *precision = b.prec;
  return QGT_OK;
}

qgt_status qgt_plan_pivot_floors(qgt_plan plan, int32_t* per_block_floors) {
  if (!plan || !per_block_floors) return fail(QGT_ERR_INVALID_ARGUMENT, "null argument");
  if (!plan->ws) return fail(QGT_ERR_INVALID_ARGUMENT, "no workspace bound");
  const size_t n = plan->blocks.size();
  hipError_t e =
      hipMemcpy(per_block_floors, plan->ws + plan->floor_off, n * sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(QGT_ERR_HIP, std::string("hipMemcpy(pivot floors): ") + hipGetErrorString(e));
  return QGT_OK;
}

qgt_status qgt_plan_block_tuning(qgt_plan plan, int32_t g, qgt_block_tuning* tuning, int32_t* source) {
  if (!plan || !tuning || !source || g < 0 || g >= (int32_t)plan->blocks.size())
    return fail(QGT_ERR_INVALID_ARGUMENT, "bad block index or null argument");
  *tuning = plan->tuning[g];
  *source = plan->tuning_src[g];
  return QGT_OK;
}

qgt_status qgt_plan_cholesky(qgt_plan plan, int32_t* mode, int32_t* source) {
  if (!plan || !mode || !source) return fail(QGT_ERR_INVALID_ARGUMENT, "null argument");
  *mode = plan->chol_host_steps ? QGT_CHOL_HOST_STEPS : QGT_CHOL_PERSISTENT;
  *source = plan->chol_mode_src;
  return QGT_OK;
}

qgt_status qgt_plan_block_factor(qgt_plan plan, int32_t g, int32_t* factor_fp32) {
  if (!plan || !factor_fp32 || g < 0 || g >= (int32_t)plan->blocks.size())
    return fail(QGT_ERR_INVALID_ARGUMENT, "bad block index or null argument");
  *factor_fp32 = plan->blocks[g].fact32;
  return QGT_OK;
}

qgt_status qgt_plan_debug_ptr(qgt_plan plan, int32_t which, int32_t index, void** ptr, int64_t* ld) {
  if (!plan || !ptr) return fail(QGT_ERR_INVALID_ARGUMENT, "null argument");
  if (!plan->ws) return fail(QGT_ERR_INVALID_ARGUMENT, "no workspace bound");
  if (ld) *ld = 0;
  if (which < 0 || which > 7) return fail(QGT_ERR_INVALID_ARGUMENT, "unknown debug buffer");
  if (which <= 2) {
    if (index < 0 || index >= plan->nprob) return fail(QGT_ERR_INVALID_ARGUMENT, "bad problem index");
    const ProbDev& p = plan->probs[index];
    const int64_t off = which == 0 ? p.mu_off : (which == 1 ? p.F_off : p.dE_off);
    *ptr = plan->ws + off;
    return QGT_OK;
  }
  if (index < 0 || index >= (int32_t)plan->blocks.size()) return fail(QGT_ERR_INVALID_ARGUMENT, "bad block index");
  const BlockDev& b = plan->blocks[index];
  if (which == 3) {
    *ptr = plan->ws + b.mat_off;
    if (ld) *ld = b.m_pad;
    return QGT_OK;
  }
  if (which == 4) {
    *ptr = plan->ws + b.pack_off;
    if (ld) *ld = b.m_pad;
    return QGT_OK;
  }
  if (which == 5) {
    *ptr = plan->ws + plan->trace_off + 8 * index;
    return QGT_OK;
  }
  if (which == 6) {
    *ptr = plan->ws + plan->cg_off + sizeof(CgScal) * index + offsetof(CgScal, est);
    return QGT_OK;
  }
  if (which == 7) {
    *ptr = plan->ws + plan->cg_off + sizeof(CgScal) * index + offsetof(CgScal, iters);
    return QGT_OK;
  }
  return fail(QGT_ERR_INVALID_ARGUMENT, "unknown debug buffer");
}

qgt_status qgt_plan_gram_timing(qgt_plan plan, int32_t precision, double* total_ms, int64_t* launches,
                                double* flops_per_launch, int32_t reset) {
  if (!plan) return fail(QGT_ERR_INVALID_ARGUMENT, "plan is null");
  if (!plan->timing) return fail(QGT_ERR_INVALID_ARGUMENT, "plan was made without timing");
  if (precision < QGT_GRAM_FP64 || precision > QGT_GRAM_BF16)
    return fail(QGT_ERR_INVALID_ARGUMENT, "precision must be FP64, FP32 or BF16");
  const int pr = precision;
  for (auto& tp : plan->tpairs[pr]) timing_collect(*plan, pr, tp);
  if (total_ms) *total_ms = plan->t_total_ms[pr];
  if (launches) *launches = plan->t_launches[pr];
  if (flops_per_launch) *flops_per_launch = plan->gram_flops[pr];
  if (reset) {
    plan->t_total_ms[pr] = 0.0;
    plan->t_launches[pr] = 0;
  }
  return QGT_OK;
}

void qgt_plan_destroy(qgt_plan plan) {
  if (!plan) return;
  {
    std::lock_guard<std::mutex> lk(g_full_mu);
    for (auto& kv : g_full_cache)
      if (kv.second->plan == plan) return;  // cached full-solve plans are freed by qgt_full_release
  }
  delete plan;
}

const char* qgt_status_string(qgt_status s) {
  switch (s) {
    case QGT_OK: return "ok";
    case QGT_ERR_INVALID_ARGUMENT: return "invalid argument";
    case QGT_ERR_UNSUPPORTED: return "unsupported";
    case QGT_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case QGT_ERR_HIP: return "HIP runtime error";
    case QGT_ERR_NOT_POSITIVE_DEFINITE: return "matrix not positive definite";
    case QGT_ERR_NOT_CONVERGED: return "refinement did not converge";
    case QGT_ERR_NON_FINITE: return "non-finite input";
    case QGT_ERR_INTERNAL: return "internal error: a device-side wait exceeded its bound";
  }
  return "unknown status";
}

const char* qgt_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// Device formation of O
// ---------------------------------------------------------------------------
size_t qgt_rbm_jacobian_workspace_bytes(int32_t n_visible, int32_t n_hidden, int64_t n_s) {
  if (n_visible < 1 || n_hidden < 1 || n_s < 1) return 0;
  Layout lay;
  lay.take((size_t)n_s * n_hidden * 16);
  return lay.bytes;
}

qgt_status qgt_rbm_jacobian(int32_t n_visible, int32_t n_hidden, const void* theta, const int8_t* x,
                            int64_t ldx, int64_t n_s, qgt_dtype o_dtype, void* O, int64_t ldo,
                            void* workspace, size_t ws_bytes, hipStream_t stream) {
  try {
    const int64_t N = n_visible, M = n_hidden;
    if (N < 1 || M < 1 || N > kJacMaxWidth || M > kJacMaxWidth)
      return fail(QGT_ERR_UNSUPPORTED, "n_visible and n_hidden must be in [1, 65535]");
    if (n_s < 1 || n_s > kJacMaxSamples) return fail(QGT_ERR_UNSUPPORTED, "n_s must be in [1, 2^24]");
    const int64_t n_p = M * N + M + N;
    if (n_p > ((int64_t)1 << 31) - 1) return fail(QGT_ERR_UNSUPPORTED, "n_p above 2^31");
    const size_t need = qgt_rbm_jacobian_workspace_bytes(n_visible, n_hidden, n_s);
    qgt_status st = jac_common_checks(theta, x, ldx, N, o_dtype, O, ldo, n_p, workspace, ws_bytes, need);
    if (st != QGT_OK) return st;
    const double2* th = (const double2*)theta;
    double2* T = (double2*)workspace;
    DenseArgs d{};
    d.x = x; d.lda = ldx; d.W = th; d.wk = 1; d.wo = N; d.bias = th + M * N; d.tg = T; d.ldt = M;
    d.n_s = n_s; d.n_o = (int32_t)M; d.n_k = (int32_t)N;
    launch_dense(0, d, stream);
    if ((st = check_launch("rbm hidden layer")) != QGT_OK) return st;
    JacArgs a{};
    jac_add_outer(a, 0, (int32_t)M, (int32_t)N, 1, 0);
    jac_add_copy(a, M * N + M, (int32_t)N, 0, 0);
    a.g[1] = T; a.ld[1] = M;
    a.x = x; a.ldx = ldx; a.O = O; a.ldo = ldo; a.n_s = n_s;
    return jac_launch_rows(a, o_dtype, stream, "rbm jacobian rows");
  } catch (...) {
    return fail(QGT_ERR_INVALID_ARGUMENT, "unexpected error");
  }
}

int64_t qgt_ffnn_n_params(const qgt_ffnn* net) {
  try {
    FfnnLayout F;
    if (ffnn_layout(net, 1, F) != QGT_OK) return -1;
    return F.n_p;
  } catch (...) {
    return -1;
  }
}

size_t qgt_ffnn_jacobian_workspace_bytes(const qgt_ffnn* net, int64_t n_s) {
  try {
    FfnnLayout F;
    if (ffnn_layout(net, n_s, F) != QGT_OK) return 0;
    return F.bytes;
  } catch (...) {
    return 0;
  }
}

qgt_status qgt_ffnn_jacobian(const qgt_ffnn* net, const void* theta, const int8_t* x, int64_t ldx,
                             int64_t n_s, qgt_dtype o_dtype, void* O, int64_t ldo, void* workspace,
                             size_t ws_bytes, hipStream_t stream) {
  try {
    FfnnLayout F;
    qgt_status st = ffnn_layout(net, n_s, F);
    if (st != QGT_OK) return st;
    const int L = net->n_layers;
    const int32_t* w = net->widths;
    st = jac_common_checks(theta, x, ldx, w[0], o_dtype, O, ldo, F.n_p, workspace, ws_bytes, F.bytes);
    if (st != QGT_OK) return st;
    const double2* th = (const double2*)theta;
    char* ws = (char*)workspace;
    auto arr = [&](int64_t off) { return off < 0 ? (double2*)nullptr : (double2*)(ws + off); };
    // forward: tanh(z^l) (times v on the last layer with a readout) and h^l
    for (int l = 1; l <= L; ++l) {
      DenseArgs d{};
      if (l == 1) { d.x = x; d.lda = ldx; }
      else { d.a = arr(F.h[l - 1]); d.lda = w[l - 1]; }
      d.W = th + F.off[l - 1]; d.wk = 1; d.wo = w[l - 1];
      d.bias = th + F.off[l - 1] + (int64_t)w[l] * w[l - 1];
      d.scale = (l == L && net->readout) ? th + F.off[L] : nullptr;
      d.tg = arr(F.tg[l]); d.h = arr(F.h[l]); d.ldt = w[l];
      d.n_s = n_s; d.n_o = w[l]; d.n_k = w[l - 1];
      launch_dense(0, d, stream);
      if ((st = check_launch("ffnn forward layer")) != QGT_OK) return st;
    }
    // backward: g^{l-1} = tanh(z^{l-1}) * (W^l)^T g^l, in place over tanh(z^{l-1})
    for (int l = L; l >= 2; --l) {
      DenseArgs d{};
      d.a = arr(F.tg[l]); d.lda = w[l];
      d.W = th + F.off[l - 1]; d.wk = w[l - 1]; d.wo = 1;
      d.tg = arr(F.tg[l - 1]); d.ldt = w[l - 1];
      d.n_s = n_s; d.n_o = w[l - 1]; d.n_k = w[l];
      launch_dense(1, d, stream);
      if ((st = check_launch("ffnn backward layer")) != QGT_OK) return st;
    }
    JacArgs a{};
    for (int l = 1; l <= L; ++l) {
      jac_add_outer(a, F.off[l - 1], w[l], w[l - 1], l, l - 1);
      a.g[l] = arr(F.tg[l]); a.v[l] = arr(F.h[l]); a.ld[l] = w[l];
    }
    if (net->readout) jac_add_copy(a, F.off[L], w[L], L, 1);
    a.x = x; a.ldx = ldx; a.O = O; a.ldo = ldo; a.n_s = n_s;
    return jac_launch_rows(a, o_dtype, stream, "ffnn jacobian rows");
  } catch (...) {
    return fail(QGT_ERR_INVALID_ARGUMENT, "unexpected error");
  }
}

int64_t qgt_cnn_n_params(const qgt_cnn* net) {
  try {
    CnnLayout F;
    if (cnn_layout(net, 1, F) != QGT_OK) return -1;
    return F.n_p;
  } catch (...) {
    return -1;
  }
}

size_t qgt_cnn_jacobian_workspace_bytes(const qgt_cnn* net, int64_t n_s) {
  try {
    CnnLayout F;
    if (cnn_layout(net, n_s, F) != QGT_OK) return 0;
    return F.bytes;
  } catch (...) {
    return 0;
  }
}

qgt_status qgt_cnn_jacobian(const qgt_cnn* net, const void* theta, const int8_t* x, int64_t ldx, int64_t n_s,
                            qgt_dtype o_dtype, void* O, int64_t ldo, void* workspace, size_t ws_bytes,
                            hipStream_t stream) {
  try {
    CnnLayout F;
    qgt_status st = cnn_layout(net, n_s, F);
    if (st != QGT_OK) return st;
    const int L = net->n_layers, C = net->channels, side = net->side;
    st = jac_common_checks(theta, x, ldx, (int64_t)side * side, o_dtype, O, ldo, F.n_p, workspace, ws_bytes,
                           F.bytes);
    if (st != QGT_OK) return st;
    const double2* th = (const double2*)theta;
    char* ws = (char*)workspace;
    auto arr = [&](int64_t off) { return off < 0 ? (double2*)nullptr : (double2*)(ws + off); };
    // forward: tanh(z^l) (on the last layer already d log psi / d z^L) and h^l
    for (int l = 1; l <= L; ++l) {
      const int cin = l == 1 ? 1 : C;
      ConvArgs c{};
      if (l == 1) { c.x = x; c.ldx = ldx; }
      else c.a = arr(F.h[l - 1]);
      c.K = th + F.off[l - 1];
      c.bias = th + F.off[l - 1] + (int64_t)C * cin * 9;
      c.tg = arr(F.tg[l]); c.h = arr(F.h[l]);
      c.n_s = n_s; c.side = side; c.cin = cin; c.cout = C; c.n_o = C; c.n_k = 9 * cin;
      launch_conv(0, c, stream);
      if ((st = check_launch("cnn forward layer")) != QGT_OK) return st;
    }
    // backward: g^{l-1} = tanh(z^{l-1}) * (kernel of layer l taken the other way, applied to g^l)
    for (int l = L; l >= 2; --l) {
      ConvArgs c{};
      c.a = arr(F.tg[l]);
      c.K = th + F.off[l - 1];
      c.tg = arr(F.tg[l - 1]);
      c.n_s = n_s; c.side = side; c.cin = C; c.cout = C; c.n_o = C; c.n_k = 9 * C;
      launch_conv(1, c, stream);
      if ((st = check_launch("cnn backward layer")) != QGT_OK) return st;
    }
    ConvDkArgs d{};
    for (int l = 1; l <= L; ++l) {
      d.layer[l - 1].g = arr(F.tg[l]);
      d.layer[l - 1].hin = l == 1 ? nullptr : arr(F.h[l - 1]);
      d.layer[l - 1].off = F.off[l - 1];
      d.layer[l - 1].cin = l == 1 ? 1 : C;
    }
    d.x = x; d.ldx = ldx; d.O = O; d.ldo = ldo; d.n_s = n_s; d.side = side; d.cout = C;
    launch_conv_dk(o_dtype == QGT_C64 ? 0 : 1, d, L, stream);
    return check_launch("cnn kernel derivatives");
  } catch (...) {
    return fail(QGT_ERR_INVALID_ARGUMENT, "unexpected error");
  }
}

}  // extern "C"
