// C ABI of the transform library: plan construction (tables, twiddles,
// workspace, tile schedules) and the four transform entry points.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "sht_internal.h"
#include "sht_plan.h"

using namespace sht;

// Workspace of sht_forward_noalloc: a static device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never uses
// this name as an address: the device address of each GPU's copy is looked
// up once per device (scratch_ptr) and passed to the kernels.
static __device__ __align__(256) unsigned char scratch[SHT_NOALLOC_WORKSPACE_BYTES];

namespace {

constexpr uint32_t kMagic = 0x53485443u;  // "SHTC"

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  if (std::getenv("SHT_LOG")) std::fprintf(stderr, "[sht] %s\n", msg.c_str());
  return code;
}

std::mutex g_live_mu;
std::set<const void*> g_live;

bool is_live(const void* p) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  return g_live.count(p) != 0;
}


}  // namespace

struct sht_plan_s {
  uint32_t magic = 0;
  int form = SHT_FORM_FP64;
  int grid = SHT_GRID_CC_POLES;
  int autotune = 0;
  int use_graph = 0;
  int reduced = 0;             // reduced transform (Sec. 4.1)
  int otf = 0;                 // Legendre kernels generate P~ from seed rows (no table kept)
  double* d_seeds = nullptr;   // per (level, m, 16-degree group): two seed rows of Kp
  long long* d_seedoff = nullptr;
  double* d_rec = nullptr;     // per (level, m, r): recurrence coefficients (A_r, B_r)
  long long* d_recoff = nullptr;
  double* d_mu = nullptr;      // per level: Kp nodes of the northern rows
  std::vector<int> jst;        // per (level, m): first latitude kept (0 if not reduced)
  int* d_jst = nullptr;
  int device = 0;
  int nlev = 0;
  int ncb = 1;                 // column blocking that fixes the workspace layout
  int ncb_fwd = 1, ncb_inv = 1;   // column blocking used by each Legendre kernel
  int fb = 8;                  // fields per zonal work item
  int sched_fwd = 0, sched_inv = 0;
  int zonal = SHT_ZONAL_AUTO;  // sht_zonal_t option
  int one_fwd = 1, one_inv = 1;   // multi-level zonal stage in one launch, per direction
  int maxN = 0;
  int nitems = 0;
  int ntiles_fwd = 0, ntiles_inv = 0;
  LevelDesc lev[SHT_MAX_LEVELS];
  size_t elem = 8;             // bytes per grid/spec scalar
  size_t grid_elems = 0, spec_elems = 0;
  size_t ws_elems = 0, table_elems = 0, table_bytes = 0, ws_bytes = 0;
  double flops = 0.0;
  double flops_kept = 0.0;     // flops the analysis kernel multiplies (reduced transform)
  bool exact = true;
  void* d_table = nullptr;      // analysis copy of the table
  void* d_table_syn = nullptr;  // synthesis copy (blocked, parity split)
  size_t table_syn_elems = 0;
  long long* d_taboff_syn = nullptr;
  void* d_ws = nullptr;
  void* d_tw = nullptr;
  double* d_w = nullptr;
  long long* d_taboff = nullptr;
  Tile* d_tiles_fwd = nullptr;
  Tile* d_tiles_inv = nullptr;
  std::vector<void*> allocs;
  size_t alloc_bytes = 0;
  // optional per-stage timing with events on the caller's stream
  int profile = 0;
  // graph replay: one captured graph per (direction, input, output)
  hipStream_t cap_stream = nullptr;
  struct GraphEntry {
    int dir;
    const void* in;
    void* out;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipEvent_t done;  // recorded after each launch; waited on before the exec is destroyed
    bool launched;
  };
  std::vector<GraphEntry> graphs;
  bool capturing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_stage;  // stage of each recorded (start, stop) pair
};

namespace {

// device bytes held by all live plans (checked against SHT_TEST_MAX_BYTES);
// plans may be built and destroyed from several threads
std::atomic<size_t> g_alloc_total{0};

// Device allocation with an optional test limit (SHT_TEST_MAX_BYTES, read at
// every call): the bytes are reserved in g_alloc_total before hipMalloc and
// released again if it fails.
int dev_alloc(sht_plan_s* P, void** out, size_t bytes) {
  const char* lim_s = std::getenv("SHT_TEST_MAX_BYTES");
  const size_t lim = lim_s ? (size_t)std::strtoull(lim_s, nullptr, 10) : 0;
  size_t cur = g_alloc_total.load();
  do {
    if (lim && cur + bytes > lim)
      return fail(SHT_ENOMEM, "device allocation of " + std::to_string(bytes) +
                                  " bytes exceeds SHT_TEST_MAX_BYTES");
  } while (!g_alloc_total.compare_exchange_weak(cur, cur + bytes));
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    g_alloc_total -= bytes;
    return fail(SHT_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  P->alloc_bytes += bytes;
  P->allocs.push_back(p);
  *out = p;
  return SHT_OK;
}

void destroy_graph_entry(sht_plan_s::GraphEntry& g) {
  // the exec may still run on the caller's stream: wait for its last launch
  if (g.launched) (void)hipEventSynchronize(g.done);
  (void)hipGraphExecDestroy(g.exec);
  (void)hipGraphDestroy(g.graph);
  if (g.done) (void)hipEventDestroy(g.done);
}

void free_plan(sht_plan_s* P) {
  for (auto& g : P->graphs) destroy_graph_entry(g);
  P->graphs.clear();
  if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
  P->cap_stream = nullptr;
  for (hipEvent_t e : P->ev_pool) (void)hipEventDestroy(e);
  P->ev_pool.clear();
  for (void* p : P->allocs) (void)hipFree(p);
  P->allocs.clear();
  g_alloc_total -= P->alloc_bytes;
  P->alloc_bytes = 0;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return SHT_OK;
  (void)hipGetLastError();
  return fail(SHT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int check_level_args(int N, int J, int I, int F, int grid) {
  if (N < 0) return fail(SHT_EINVAL, "N must be >= 0");
  if (F < 1) return fail(SHT_EINVAL, "nfields must be >= 1");
  if (!grid_args_ok(J, grid))
    return fail(SHT_EINVAL, grid == SHT_GRID_CC_POLES ? "J must be >= 2 on the CC grid with poles"
                                                     : (grid == SHT_GRID_FEJER2 || grid == SHT_GRID_FEJER1 ||
                                                                grid == SHT_GRID_GAUSS
                                                            ? "J must be >= 1"
                                                                                : "unknown grid kind"));
  if (I < 2 * N + 1) return fail(SHT_EINVAL, "I must be >= 2N+1 (no retained wavenumber may alias)");
  if (I > SHT_MAX_I) return fail(SHT_EINVAL, "I exceeds the supported maximum 4096");
  int rad[SHT_MAX_RADICES], nrad;
  if (!factor_radices(I, rad, &nrad)) return fail(SHT_EINVAL, "I must factor into 2, 3 and 5");
  return SHT_OK;
}

int autotune(sht_plan_s* P);
bool blocking_ok(const sht_plan_s* P, bool analysis, int c);

int build_plan(int nlev, const int* Nv, const int* Jv, const int* Iv, const int* Fv,
               const sht_options* opts, sht_plan_t* out) {
  if (!out) return fail(SHT_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (nlev < 1 || nlev > SHT_MAX_LEVELS) return fail(SHT_EINVAL, "nlevels must be 1..8");
  if (!Nv || !Jv || !Iv || !Fv) return fail(SHT_EINVAL, "level arrays must not be NULL");
  sht_options o{SHT_GRID_CC_POLES, SHT_FORM_FP64, 0, 0, 0, 0, SHT_ZONAL_AUTO};
  if (opts) o = *opts;
  if (o.form < SHT_FORM_FP64 || o.form > SHT_FORM_BF16X6) return fail(SHT_EINVAL, "unknown form");
  if (o.zonal < SHT_ZONAL_AUTO || o.zonal > SHT_ZONAL_PER_LENGTH) return fail(SHT_EINVAL, "unknown zonal launch mode");
  if (o.otf && (o.reduced || o.autotune)) return fail(SHT_EINVAL, "otf cannot be combined with reduced or autotune");
  for (int l = 0; l < nlev; ++l) {
    int rc = check_level_args(Nv[l], Jv[l], Iv[l], Fv[l], o.grid);
    if (rc) return rc;
  }

  sht_plan_s* P = new (std::nothrow) sht_plan_s();
  if (!P) return fail(SHT_ENOMEM, "host allocation failed");
  P->form = o.form;
  P->grid = o.grid;
  P->autotune = o.autotune;
  P->use_graph = o.use_graph;
  P->reduced = o.reduced != 0;
  P->otf = o.otf != 0;
  P->zonal = o.zonal;
  P->one_fwd = P->one_inv = o.zonal != SHT_ZONAL_PER_LENGTH;
  if (o.zonal == SHT_ZONAL_AUTO && nlev > 1) {
    // without a timing, one launch only where its kernel keeps everything in
    // registers (the autotuner, if asked for, times both and decides)
    P->one_fwd = !zonal_one_launch_spills(o.form, true);
    P->one_inv = !zonal_one_launch_spills(o.form, false);
  }
  P->nlev = nlev;
  P->elem = o.form == SHT_FORM_FP64 ? 8 : 4;
  int rc = hip_check(hipGetDevice(&P->device), "hipGetDevice");
  if (rc) {
    delete P;
    return rc;
  }
  P->ncb = choose_ncb(o.form, nlev, Nv, Jv, Fv);
  const int BN = 16 * P->ncb;
  int FB = zonal_fields_per_block(o.form, nlev, Nv[0], Jv[0], Iv[0], Fv[0]);
  if (FB > 8) {
    // the wide blocking runs only in the fixed-length kernel, whose
    // workspace offsets are 32-bit
    const long long Cp = roundup(2LL * Fv[0], std::lcm(BN, 2 * FB));
    const long long Kp = roundup((Jv[0] + 1) / 2, SHT_K_PAD);
    if (!zonal_offsets_fit(ws_plane(Kp, Cp), (long long)P->elem)) FB = 8;
  }
  P->fb = FB;

  // ---- level descriptors and sizes ----
  Layout Y;
  layout_levels(nlev, Nv, Jv, Iv, Fv, BN, FB, P->lev, &Y);
  const long long item = Y.items, goff = Y.grid, soff = Y.spec, woff = Y.ws, moff = Y.nm_total;
  const std::vector<long long>&taboff = Y.taboff, &taboff_syn = Y.taboff_syn, &seedoff = Y.seedoff,
                           &recoff = Y.recoff;
  const long long tab = Y.tab, tabs = Y.tabs, seeds_total = Y.seeds, rec_total = Y.rec;
  for (int l = 0; l < nlev; ++l) {
    const LevelDesc& L = P->lev[l];
    P->maxN = std::max(P->maxN, L.N);
    P->flops += 2.0 * L.Jh * (double)(L.N + 1) * (L.N + 2) * L.F;
    // Gauss-Legendre on J nodes is exact to degree 2J-1, the CC rules to J-1
    if (o.grid == SHT_GRID_GAUSS ? L.J < L.N + 1 : L.J < 2 * L.N + 1) P->exact = false;
  }
  if (item > 0x7fffffff) {
    delete P;
    return fail(SHT_EINVAL, "too many zonal work items");
  }
  P->nitems = (int)item;
  P->grid_elems = (size_t)goff;
  P->spec_elems = (size_t)soff;
  P->ws_elems = (size_t)woff;
  // with generated P~ no table copy is kept (seed rows only)
  P->table_elems = P->otf ? 0 : (size_t)tab;
  P->table_syn_elems = P->otf ? 0 : (size_t)tabs;
  // bytes per table element (the split form reads the FP32 copies)
  const size_t tel = P->elem;
  P->table_bytes = (P->table_elems + P->table_syn_elems) * tel;
  P->ws_bytes = P->ws_elems * P->elem;

  // ---- host tables ----
  std::vector<unsigned char> htab(P->table_elems * tel), htabs(P->table_syn_elems * tel);
  P->jst.assign((size_t)moff, 0);
  std::vector<double> hw;
  std::vector<std::vector<unsigned char>> htw(nlev);
  size_t tw_total = 0;
  std::vector<size_t> tw_off(nlev), w_off(nlev), mu_off(nlev);
  size_t w_total = 0, mu_total = 0;
  std::vector<double> hseeds(P->otf ? (size_t)seeds_total : 0), hrec(P->otf ? (size_t)rec_total : 0), hmu;
  for (int l = 0; l < nlev; ++l) {
    LevelDesc& L = P->lev[l];
    std::vector<double> mu(L.J), sint(L.J), w(L.J);
    grid_nodes(L.J, o.grid, mu.data(), sint.data());
    grid_weights(L.J, o.grid, w.data());
    w_off[l] = w_total;
    w_total += L.Jh;
    hw.insert(hw.end(), w.begin(), w.begin() + L.Jh);
    if (P->otf) {
      mu_off[l] = mu_total;
      mu_total += L.Kp;
      for (int j = 0; j < L.Kp; ++j) hmu.push_back(j < L.Jh ? mu[j] : 0.0);
      // P~_n = a_n (mu P~_{n-1} - P~_{n-2} / a_{n-1}), a_n = sqrt((4n^2-1)/(n^2-m^2))
      for (int m = 0; m <= L.N; ++m) {
        double* rc2 = hrec.data() + recoff[L.m_base + m];
        long double aprev = 0.0L;
        for (int r = 0; r <= L.N - m; ++r) {
          const long double n = (long double)(m + r), mm = (long double)m * m;
          const long double a = r >= 1 ? sqrtl((4.0L * n * n - 1.0L) / (n * n - mm)) : 0.0L;
          rc2[2 * r] = (double)a;
          rc2[2 * r + 1] = r >= 2 ? (double)(a / aprev) : 0.0;
          aprev = a;
        }
      }
    }
    const long long* to = taboff.data() + L.m_base;
    const long long* ts = taboff_syn.data() + L.m_base;
    if (o.form == SHT_FORM_FP64)
      fill_table_level<double>(L, mu.data(), sint.data(), P->otf ? nullptr : reinterpret_cast<double*>(htab.data()), to,
                               P->otf ? nullptr : reinterpret_cast<double*>(htabs.data()), ts,
                               P->reduced ? P->jst.data() + L.m_base : nullptr,
                               P->otf ? hseeds.data() : nullptr, seedoff.data() + L.m_base);
    else
      fill_table_level<float>(L, mu.data(), sint.data(), P->otf ? nullptr : reinterpret_cast<float*>(htab.data()), to,
                              P->otf ? nullptr : reinterpret_cast<float*>(htabs.data()), ts,
                              P->reduced ? P->jst.data() + L.m_base : nullptr, P->otf ? hseeds.data() : nullptr,
                              seedoff.data() + L.m_base);
    // twiddles exp(-2 pi i k / I)
    const size_t cs = 2 * P->elem;
    htw[l].resize((size_t)L.I * cs);
    for (int k = 0; k < L.I; ++k) {
      const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)k / (long double)L.I;
      const long double c = cosl(ang), s = -sinl(ang);
      if (o.form == SHT_FORM_FP64) {
        double v[2] = {(double)c, (double)s};
        std::memcpy(&htw[l][k * cs], v, cs);
      } else {
        float v[2] = {(float)c, (float)s};
        std::memcpy(&htw[l][k * cs], v, cs);
      }
    }
    tw_off[l] = tw_total;
    tw_total += roundup((long long)htw[l].size(), 256);
  }

  // ---- tile schedules (default; the autotuner may replace them) ----
  // the kernels keep their whole output tile in registers: where the
  // plan's blocking is wider than a kernel takes, use the widest blocking it
  // supports that divides every level's row length
  for (int dir = 0; dir < 2; ++dir) {
    int& ncb = dir == 0 ? P->ncb_fwd : P->ncb_inv;
    ncb = P->ncb;
    if (ncb <= max_ncb(o.form, dir == 0)) continue;
    for (int c : {8, 5, 4, 2, 1}) {
      if (c > max_ncb(o.form, dir == 0)) continue;
      bool ok = true;
      for (int l = 0; l < nlev; ++l)
        if (P->lev[l].Cp % (16 * c)) ok = false;
      if (ok) {
        ncb = c;
        break;
      }
    }
  }
  // small plans: where a direction's tiles would not give every compute
  // unit two workgroups, narrower column tiles (more of them) are taken, as
  // long as a narrower blocking is admissible (blocking_ok); the idle slots
  // that even out the XCD chunks of a tile list do not count
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess || ncu <= 0)
      ncu = 256;
    auto real_tiles = [&](bool analysis, int c) {
      size_t n = 0;
      for (const Tile& t : build_tiles(P->form, nlev, P->lev, P->jst.data(), analysis, c, 0)) n += t.level >= 0;
      return n;
    };
    for (int dir = 0; dir < 2; ++dir) {
      int& ncb = dir == 0 ? P->ncb_fwd : P->ncb_inv;
      while (real_tiles(dir == 0, ncb) < 2 * (size_t)ncu) {
        int next = 0;
        for (int c : {8, 5, 4, 2, 1})
          if (c < ncb && blocking_ok(P, dir == 0, c)) {
            next = c;
            break;
          }
        if (!next) break;
        ncb = next;
      }
    }
  }
  // flops kept by the reduced transform (whole analysis blocks left out)
  P->flops_kept = 0.0;
  for (int l = 0; l < nlev; ++l) {
    const LevelDesc& L = P->lev[l];
    const int kb = o.form == SHT_FORM_FP64 ? 16 : 32;
    for (int m = 0; m <= L.N; ++m)
      P->flops_kept += 4.0 * (L.N - m + 1) * L.F * (double)(L.Jh - P->jst[L.m_base + m] / kb * kb);
  }
  std::vector<Tile> sf = build_tiles(P->form, P->nlev, P->lev, P->jst.data(), true, P->ncb_fwd, 0),
                    si = build_tiles(P->form, P->nlev, P->lev, P->jst.data(), false, P->ncb_inv, 0);
  P->ntiles_fwd = (int)sf.size();
  P->ntiles_inv = (int)si.size();

  // ---- device buffers ----
  void *dtw = nullptr, *dw = nullptr, *dto = nullptr, *dtf = nullptr, *dti = nullptr, *dtos = nullptr,
       *djs = nullptr;
  if ((rc = dev_alloc(P, &P->d_table, htab.size())) ||
      (rc = dev_alloc(P, &P->d_table_syn, htabs.size())) ||
      (rc = dev_alloc(P, &dtos, taboff_syn.size() * sizeof(long long))) ||
      (rc = dev_alloc(P, &P->d_ws, P->ws_bytes)) ||
      (rc = dev_alloc(P, &dtw, tw_total)) ||
      (rc = dev_alloc(P, &dw, w_total * sizeof(double))) ||
      (rc = dev_alloc(P, &dto, taboff.size() * sizeof(long long))) ||
      (rc = dev_alloc(P, &dtf, sf.size() * sizeof(Tile))) ||
      (rc = dev_alloc(P, &dti, si.size() * sizeof(Tile))) ||
      (rc = dev_alloc(P, &djs, P->jst.size() * sizeof(int)))) {
    free_plan(P);
    delete P;
    return rc;
  }
  P->d_tw = dtw;
  P->d_w = static_cast<double*>(dw);
  P->d_taboff = static_cast<long long*>(dto);
  P->d_taboff_syn = static_cast<long long*>(dtos);
  P->d_tiles_fwd = static_cast<Tile*>(dtf);
  P->d_tiles_inv = static_cast<Tile*>(dti);
  P->d_jst = static_cast<int*>(djs);
  for (int l = 0; l < nlev; ++l) {
    P->lev[l].tw = static_cast<unsigned char*>(dtw) + tw_off[l];
    P->lev[l].wrow = P->d_w + w_off[l];
  }
  rc = hip_check(hipMemcpy(P->d_table, htab.data(), htab.size(), hipMemcpyHostToDevice), "upload table");
  if (!rc)
    rc = hip_check(hipMemcpy(P->d_table_syn, htabs.data(), htabs.size(), hipMemcpyHostToDevice), "upload table");
  if (!rc)
    rc = hip_check(hipMemcpy(dtos, taboff_syn.data(), taboff_syn.size() * sizeof(long long), hipMemcpyHostToDevice),
                   "upload table offsets");
  if (!rc) rc = hip_check(hipMemset(P->d_ws, 0, P->ws_bytes), "clear workspace");
  for (int l = 0; l < nlev && !rc; ++l)
    rc = hip_check(hipMemcpy(static_cast<unsigned char*>(dtw) + tw_off[l], htw[l].data(), htw[l].size(),
                             hipMemcpyHostToDevice),
                   "upload twiddles");
  if (!rc) rc = hip_check(hipMemcpy(dw, hw.data(), w_total * sizeof(double), hipMemcpyHostToDevice), "upload weights");
  if (!rc)
    rc = hip_check(hipMemcpy(dto, taboff.data(), taboff.size() * sizeof(long long), hipMemcpyHostToDevice),
                   "upload table offsets");
  if (!rc) rc = hip_check(hipMemcpy(dtf, sf.data(), sf.size() * sizeof(Tile), hipMemcpyHostToDevice), "upload tiles");
  if (!rc) rc = hip_check(hipMemcpy(dti, si.data(), si.size() * sizeof(Tile), hipMemcpyHostToDevice), "upload tiles");
  if (!rc)
    rc = hip_check(hipMemcpy(djs, P->jst.data(), P->jst.size() * sizeof(int), hipMemcpyHostToDevice),
                   "upload latitude starts");
  if (!rc && P->otf) {
    void *dsd = nullptr, *dso = nullptr, *drc = nullptr, *dro = nullptr, *dmu = nullptr;
    if (!(rc = dev_alloc(P, &dsd, hseeds.size() * sizeof(double))) &&
        !(rc = dev_alloc(P, &dso, seedoff.size() * sizeof(long long))) &&
        !(rc = dev_alloc(P, &drc, hrec.size() * sizeof(double))) &&
        !(rc = dev_alloc(P, &dro, recoff.size() * sizeof(long long))) &&
        !(rc = dev_alloc(P, &dmu, hmu.size() * sizeof(double)))) {
      P->d_seeds = static_cast<double*>(dsd);
      P->d_seedoff = static_cast<long long*>(dso);
      P->d_rec = static_cast<double*>(drc);
      P->d_recoff = static_cast<long long*>(dro);
      P->d_mu = static_cast<double*>(dmu);
      for (int l = 0; l < nlev; ++l) P->lev[l].murow = P->d_mu + mu_off[l];
      rc = hip_check(hipMemcpy(dsd, hseeds.data(), hseeds.size() * sizeof(double), hipMemcpyHostToDevice),
                     "upload seeds");
      if (!rc)
        rc = hip_check(hipMemcpy(dso, seedoff.data(), seedoff.size() * sizeof(long long), hipMemcpyHostToDevice),
                       "upload seed offsets");
      if (!rc)
        rc = hip_check(hipMemcpy(drc, hrec.data(), hrec.size() * sizeof(double), hipMemcpyHostToDevice),
                       "upload recurrence");
      if (!rc)
        rc = hip_check(hipMemcpy(dro, recoff.data(), recoff.size() * sizeof(long long), hipMemcpyHostToDevice),
                       "upload recurrence offsets");
      if (!rc)
        rc = hip_check(hipMemcpy(dmu, hmu.data(), hmu.size() * sizeof(double), hipMemcpyHostToDevice), "upload nodes");
    }
  }
  if (!rc) rc = hip_check(hipDeviceSynchronize(), "plan synchronize");
  if (!rc && o.autotune) rc = autotune(P);
  if (rc) {
    free_plan(P);
    delete P;
    return rc;
  }
  P->magic = kMagic;
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert(P);
  }
  *out = P;
  return SHT_OK;
}

int check_plan(sht_plan_t p) {
  if (!p) return fail(SHT_EINVAL, "plan is NULL");
  if (!is_live(p) || p->magic != kMagic) return fail(SHT_ESTATE, "plan handle is not live (destroyed?)");
  return SHT_OK;
}

int check_ptr(const void* p, const char* name, int align = 16) {
  if (!p) return fail(SHT_EINVAL, std::string(name) + " must not be NULL");
  if (reinterpret_cast<uintptr_t>(p) % align)
    return fail(SHT_EINVAL, std::string(name) + " must be " + std::to_string(align) + "-byte aligned");
  return SHT_OK;
}

FftArgs fft_args(const sht_plan_s* P, const void* src, void* dst, int use_w, int use_inv_I, double mscale) {
  FftArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nlev = P->nlev;
  a.nitems = P->nitems;
  for (int l = 0; l < P->nlev; ++l) a.lev[l] = P->lev[l];
  a.src = src;
  a.dst = dst;
  a.use_w = use_w;
  a.use_inv_I = use_inv_I;
  a.mscale = mscale;
  a.fb = P->fb;
  a.jstart = P->reduced ? P->d_jst : nullptr;  // null: no latitude left out
  return a;
}

GemmArgs gemm_args(const sht_plan_s* P, bool analysis, const void* spec_in, void* spec_out) {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.nlev = P->nlev;
  for (int l = 0; l < P->nlev; ++l) g.lev[l] = P->lev[l];
  g.ntiles = analysis ? P->ntiles_fwd : P->ntiles_inv;
  g.tiles = analysis ? P->d_tiles_fwd : P->d_tiles_inv;
  g.tab_off = analysis ? P->d_taboff : P->d_taboff_syn;
  g.table = analysis ? P->d_table : P->d_table_syn;
  g.jstart = P->d_jst;
  g.spec_in = spec_in;
  g.spec_out = spec_out;
  g.ws = P->d_ws;
  g.seeds = P->d_seeds;
  g.seed_off = P->d_seedoff;
  g.rec = P->d_rec;
  g.rec_off = P->d_recoff;
  return g;
}

// Stage ids for profiling.
enum { ST_ZONAL_A = 0, ST_LEG_A = 1, ST_LEG_S = 2, ST_ZONAL_S = 3, ST_COUNT = 4 };

hipEvent_t next_event(sht_plan_s* P) {
  if (P->ev_used == P->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    P->ev_pool.push_back(e);
  }
  return P->ev_pool[P->ev_used++];
}

void prof_mark(sht_plan_s* P, void* stream, int stage, bool start) {
  if (!P->profile || P->capturing) return;
  hipEvent_t e = next_event(P);
  if (!e) return;
  (void)hipEventRecord(e, static_cast<hipStream_t>(stream));
  if (start) P->ev_stage.push_back(stage);
}

// grid -> spec through the zonal analysis (row scale and m scale given);
// ws is the workspace to use (the plan's, or the static scratch)
int run_analysis(sht_plan_s* P, const void* grid, void* spec, void* stream, int use_w, int use_inv_I,
                 double mscale, void* ws) {
  FftArgs a = fft_args(P, grid, ws, use_w, use_inv_I, mscale);
  a.one_launch = P->one_fwd;
  prof_mark(P, stream, ST_ZONAL_A, true);
  int e = launch_zonal(P->form, true, a, P->maxN, stream);
  prof_mark(P, stream, ST_ZONAL_A, false);
  if (e) return hip_check((hipError_t)e, "zonal analysis launch");
  GemmArgs g = gemm_args(P, true, nullptr, spec);
  g.ws = ws;
  prof_mark(P, stream, ST_LEG_A, true);
  e = launch_legendre(P->form, true, g, P->ncb_fwd, P->otf != 0, stream);
  prof_mark(P, stream, ST_LEG_A, false);
  if (e) return hip_check((hipError_t)e, "Legendre analysis launch");
  return SHT_OK;
}

int run_synthesis(sht_plan_s* P, const void* spec, void* grid, void* stream, int use_w, int use_inv_I,
                  double mscale) {
  GemmArgs g = gemm_args(P, false, spec, nullptr);
  prof_mark(P, stream, ST_LEG_S, true);
  int e = launch_legendre(P->form, false, g, P->ncb_inv, P->otf != 0, stream);
  prof_mark(P, stream, ST_LEG_S, false);
  if (e) return hip_check((hipError_t)e, "Legendre synthesis launch");
  FftArgs a = fft_args(P, P->d_ws, grid, use_w, use_inv_I, mscale);
  a.one_launch = P->one_inv;
  prof_mark(P, stream, ST_ZONAL_S, true);
  e = launch_zonal(P->form, false, a, P->maxN, stream);
  prof_mark(P, stream, ST_ZONAL_S, false);
  if (e) return hip_check((hipError_t)e, "zonal synthesis launch");
  return SHT_OK;
}

enum { DIR_FWD = 0, DIR_INV = 1, DIR_FWD_ADJ = 2, DIR_INV_ADJ = 3 };

int run_eager(sht_plan_s* P, int dir, const void* in, void* out, void* stream) {
  switch (dir) {
    case DIR_FWD: return run_analysis(P, in, out, stream, 1, 1, 1.0, P->d_ws);
    case DIR_INV: return run_synthesis(P, in, out, stream, 0, 0, 1.0);
    case DIR_FWD_ADJ: return run_synthesis(P, in, out, stream, 1, 1, 0.5);
    default: return run_analysis(P, in, out, stream, 0, 0, 2.0, P->d_ws);
  }
}

// With use_graph, the first call for a (direction, input, output) triple
// runs eagerly and records its launches into a hipGraph on a private
// stream; later calls replay the graph on the caller's stream.
int run_dir(sht_plan_s* P, int dir, const void* in, void* out, void* stream) {
  if (!P->use_graph) return run_eager(P, dir, in, out, stream);
  for (auto& g : P->graphs)
    if (g.dir == dir && g.in == in && g.out == out) {
      int rc = hip_check(hipGraphLaunch(g.exec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
      if (rc) return rc;
      rc = hip_check(hipEventRecord(g.done, static_cast<hipStream_t>(stream)), "record graph event");
      if (!rc) g.launched = true;
      return rc;
    }
  int rc = run_eager(P, dir, in, out, stream);
  if (rc) return rc;
  if (!P->cap_stream && (rc = hip_check(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking),
                                        "create capture stream")))
    return rc;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  P->capturing = true;
  rc = hip_check(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  if (!rc) {
    int rc2 = run_eager(P, dir, in, out, P->cap_stream);
    rc = hip_check(hipStreamEndCapture(P->cap_stream, &graph), "end capture");
    if (!rc) rc = rc2;
  }
  P->capturing = false;
  if (!rc) rc = hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate graph");
  hipEvent_t done = nullptr;
  if (!rc) rc = hip_check(hipEventCreateWithFlags(&done, hipEventDisableTiming), "create graph event");
  if (rc) {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  // at most 16 cached graphs: the oldest goes once its last launch is done
  if (P->graphs.size() >= 16) {
    destroy_graph_entry(P->graphs.front());
    P->graphs.erase(P->graphs.begin());
  }
  P->graphs.push_back({dir, in, out, graph, exec, done, false});
  return SHT_OK;
}

// ---- allocation-free analysis ----

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (dev must be the
// current device); looked up on the first call per device.
int scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SHT_EINVAL, "device id out of range for the static workspace");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    int rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    if (!p) return fail(SHT_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SHT_OK;
}

// The analysis with the workspace in the static array.  The Legendre
// analysis reads the padding rows ceil(J/2) <= j < Kp of every wavenumber's
// workspace region (their table entries are zero), and an earlier call, of
// this or another plan, may have left any value there (NaN included): they
// are cleared first by a fill kernel on the same stream.  No events, graphs
// or allocations.
int run_forward_noalloc(sht_plan_s* P, const void* grid, void* spec, void* stream) {
  if (P->ws_bytes > SHT_NOALLOC_WORKSPACE_BYTES)
    return fail(SHT_EINVAL, "the plan's workspace (" + std::to_string(P->ws_bytes) +
                                " bytes) exceeds the static workspace of sht_forward_noalloc (" +
                                std::to_string((size_t)SHT_NOALLOC_WORKSPACE_BYTES) + " bytes)");
  int dev = -1;
  int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev != P->device)
    return fail(SHT_EINVAL, "the plan was built on device " + std::to_string(P->device) +
                                " but the current device is " + std::to_string(dev));
  void* ws = nullptr;
  if ((rc = scratch_ptr(dev, &ws))) return rc;
  for (int l = 0; l < P->nlev; ++l) {
    const LevelDesc& L = P->lev[l];
    // an analysis row holds 2 Cp elements (both parities), Cp a multiple of
    // 16; the regions are 2 wplane elements apart, wplane a multiple of 16
    const long long row16 = 2LL * L.Cp * (long long)P->elem / 16;
    const long long region16 = 2LL * L.wplane * (long long)P->elem / 16;
    const int e = launch_clear_span(static_cast<unsigned char*>(ws) + L.ws_off * (long long)P->elem,
                                    (long long)(L.N + 1), region16, row16 * L.Jh, row16 * (L.Kp - L.Jh), stream);
    if (e) return hip_check((hipError_t)e, "workspace clear launch");
  }
  const int saved_profile = P->profile;  // profiling would create events
  P->profile = 0;
  rc = run_analysis(P, grid, spec, stream, 1, 1, 1.0, ws);
  P->profile = saved_profile;
  return rc;
}

// ---- autotuner ----

std::string tune_path() {
  if (const char* e = std::getenv("SHT_TUNE_CACHE")) return e;
  const char* h = std::getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/sht_tune.txt";
}

// The key pins everything a cached choice depends on: device architecture,
// HIP runtime version, the tuner's version, form, every level's sizes and the
// workspace layout (row length Cp, fields per zonal item).
std::string tune_key(const sht_plan_s* P) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) arch = prop.gcnArchName;
  for (auto& ch : arch)
    if (ch == ' ') ch = '_';
  int rt = 0;
  (void)hipRuntimeGetVersion(&rt);
  std::string k = arch + " hip" + std::to_string(rt) + " v3 form" + std::to_string(P->form) + " fb" +
                  std::to_string(P->fb) + " lev" + std::to_string(P->nlev);
  for (int l = 0; l < P->nlev; ++l)
    k += " " + std::to_string(P->lev[l].N) + "," + std::to_string(P->lev[l].J) + "," + std::to_string(P->lev[l].I) +
         "," + std::to_string(P->lev[l].F) + "," + std::to_string(P->lev[l].Cp);
  return k;
}

// A column blocking c (16-column units) is admissible for a direction when
// the kernel takes it and it tiles every level's workspace row exactly with
// no tile wholly past the last field.
bool blocking_ok(const sht_plan_s* P, bool analysis, int c) {
  if (c < 1 || c > max_ncb(P->form, analysis)) return false;
  for (int l = 0; l < P->nlev; ++l)
    if (P->lev[l].Cp % (16 * c) || roundup(2LL * P->lev[l].F, 16LL * c) != P->lev[l].Cp) return false;
  return true;
}

bool tune_lookup(const std::string& key, int v[6]) {
  FILE* f = std::fopen(tune_path().c_str(), "r");
  if (!f) return false;
  char line[4096];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    std::string l(line);
    size_t bar = l.find('|');
    if (bar == std::string::npos || l.substr(0, bar) != key) continue;
    found = std::sscanf(l.c_str() + bar + 1, "%d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == 6;
  }
  std::fclose(f);
  return found;
}

void tune_store(const std::string& key, const int v[6]) {
  FILE* f = std::fopen(tune_path().c_str(), "a");
  if (!f) return;  // the cache is optional
  std::fprintf(f, "%s|%d %d %d %d %d %d\n", key.c_str(), v[0], v[1], v[2], v[3], v[4], v[5]);
  std::fclose(f);
}

int upload_tiles(sht_plan_s* P, bool analysis, const std::vector<Tile>& t) {
  Tile** slot = analysis ? &P->d_tiles_fwd : &P->d_tiles_inv;
  int* cnt = analysis ? &P->ntiles_fwd : &P->ntiles_inv;
  if ((size_t)*cnt < t.size()) {
    void* p = nullptr;
    int rc = dev_alloc(P, &p, t.size() * sizeof(Tile));
    if (rc) return rc;
    *slot = static_cast<Tile*>(p);  // the old buffer is freed with the plan
  }
  *cnt = (int)t.size();
  return hip_check(hipMemcpy(*slot, t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice), "upload tiles");
}

// Time the Legendre kernels for every column blocking that keeps the
// workspace layout and both tile orders, and (multi-level plans) the zonal
// stage in one launch and per FFT length; keep the fastest per direction.
// Cache line: ncb and order of the analysis, the same of the synthesis,
// one-launch zonal analysis and synthesis (0/1).
int autotune(sht_plan_s* P) {
  const std::string key = tune_key(P);
  int v[6];
  // a cached entry is used only if it passes the same filter as the search
  // (a stale or foreign line could otherwise leave columns uncomputed)
  // (the plan's default blocking, which the search keeps when no candidate
  // passes, is also accepted)
  const bool cached = tune_lookup(key, v) && (v[0] == P->ncb_fwd || blocking_ok(P, true, v[0])) &&
                      (v[2] == P->ncb_inv || blocking_ok(P, false, v[2])) && (v[1] == 0 || v[1] == 1) &&
                      (v[3] == 0 || v[3] == 1) && (v[4] == 0 || v[4] == 1) && (v[5] == 0 || v[5] == 1);
  if (!cached) {
    const int all64[] = {1, 2, 4, 8}, all32[] = {1, 2, 4, 5, 8, 10};
    const int* all = P->form == SHT_FORM_FP64 ? all64 : all32;
    const int na = P->form == SHT_FORM_FP64 ? 4 : 6;
    void* spec = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SHT_OK;
    if ((rc = hip_check(hipMalloc(&spec, P->spec_elems * P->elem + 16), "tune alloc"))) return rc;
    (void)hipMemset(spec, 0, P->spec_elems * P->elem);
    (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int saved_profile = P->profile;
    P->profile = 0;
    for (int dir = 0; dir < 2 && !rc; ++dir) {
      const bool analysis = dir == 0;
      float best = 1e30f;
      int bc = analysis ? P->ncb_fwd : P->ncb_inv, bs = 0;
      for (int k = 0; k < na; ++k)
        for (int sched = 0; sched < 2 && !rc; ++sched) {
          const int c = all[k];
          if (!blocking_ok(P, analysis, c)) continue;
          std::vector<Tile> t = build_tiles(P->form, P->nlev, P->lev, P->jst.data(), analysis, c, sched);
          Tile* dt = nullptr;
          if ((rc = hip_check(hipMalloc(reinterpret_cast<void**>(&dt), t.size() * sizeof(Tile)), "tune alloc"))) break;
          (void)hipMemcpy(dt, t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice);
          GemmArgs g = gemm_args(P, analysis, spec, spec);
          g.tiles = dt;
          g.ntiles = (int)t.size();
          int e = launch_legendre(P->form, analysis, g, c, false, st);
          (void)hipEventRecord(e0, st);
          for (int r = 0; r < 3 && !e; ++r) e = launch_legendre(P->form, analysis, g, c, false, st);
          (void)hipEventRecord(e1, st);
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          (void)hipFree(dt);
          if (e) {
            rc = hip_check((hipError_t)e, "tune launch");
            break;
          }
          if (ms < best) {
            best = ms;
            bc = c;
            bs = sched;
          }
        }
      v[2 * dir] = bc;
      v[2 * dir + 1] = bs;
    }
    // zonal stage of a multi-level plan: one launch over all levels against
    // one per FFT length (the same when the levels do not allow one launch;
    // ties keep one launch)
    v[4] = v[5] = 1;
    if (!rc && P->nlev > 1) {
      void* grid = nullptr;
      rc = hip_check(hipMalloc(&grid, P->grid_elems * P->elem + 16), "tune alloc");
      if (!rc) rc = hip_check(hipMemset(grid, 0, P->grid_elems * P->elem), "tune clear");
      for (int dir = 0; dir < 2 && !rc; ++dir) {
        const bool analysis = dir == 0;
        float best = 1e30f;
        for (int one = 1; one >= 0 && !rc; --one) {
          FftArgs a = analysis ? fft_args(P, grid, P->d_ws, 1, 1, 1.0) : fft_args(P, P->d_ws, grid, 0, 0, 1.0);
          a.one_launch = one;
          int e = launch_zonal(P->form, analysis, a, P->maxN, st);
          (void)hipEventRecord(e0, st);
          for (int r = 0; r < 3 && !e; ++r) e = launch_zonal(P->form, analysis, a, P->maxN, st);
          (void)hipEventRecord(e1, st);
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (e) {
            rc = hip_check((hipError_t)e, "tune zonal launch");
            break;
          }
          if (ms < best) {
            best = ms;
            v[4 + dir] = one;
          }
        }
      }
      if (grid) (void)hipFree(grid);
    }
    P->profile = saved_profile;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    (void)hipFree(spec);
    if (rc) return rc;
    tune_store(key, v);
  }
  P->ncb_fwd = v[0];
  P->sched_fwd = v[1];
  P->ncb_inv = v[2];
  P->sched_inv = v[3];
  if (P->zonal == SHT_ZONAL_AUTO) {
    P->one_fwd = v[4];
    P->one_inv = v[5];
  }
  int rc = upload_tiles(P, true, build_tiles(P->form, P->nlev, P->lev, P->jst.data(), true, P->ncb_fwd, P->sched_fwd));
  if (!rc)
    rc = upload_tiles(P, false,
                      build_tiles(P->form, P->nlev, P->lev, P->jst.data(), false, P->ncb_inv, P->sched_inv));
  return rc;
}

}  // namespace

extern "C" {

const char* sht_last_error(void) { return g_err.c_str(); }

int sht_device_bytes(size_t* out) {
  if (!out) return fail(SHT_EINVAL, "out must not be NULL");
  *out = g_alloc_total.load();
  return SHT_OK;
}

int sht_spec_retruncate(int N_in, int N_out, int nfields, int dbl, const void* spec_in, void* spec_out,
                        void* stream) {
  if (N_in < 0 || N_out < 0 || nfields < 1) return fail(SHT_EINVAL, "need N_in, N_out >= 0 and nfields >= 1");
  if (N_out > 65534 || nfields > 65535) return fail(SHT_EINVAL, "N_out or nfields too large");
  int rc = check_ptr(spec_in, "spec_in");
  if (!rc) rc = check_ptr(spec_out, "spec_out");
  if (rc) return rc;
  if (spec_in == spec_out) return fail(SHT_EINVAL, "spec_in and spec_out must not overlap");
  return hip_check((hipError_t)launch_retruncate(N_in, N_out, nfields, dbl != 0, spec_in, spec_out, stream),
                   "retruncate launch");
}

int sht_grid_product(long long n, int dbl, const void* a, const void* b, void* out, void* stream) {
  if (n < 1) return fail(SHT_EINVAL, "n must be >= 1");
  int rc = check_ptr(a, "a");
  if (!rc) rc = check_ptr(b, "b");
  if (!rc) rc = check_ptr(out, "out");
  if (rc) return rc;
  return hip_check((hipError_t)launch_product(n, dbl != 0, a, b, out, stream), "product launch");
}

int sht_spec_laplacian(int N, int nfields, int dbl, double scale, const void* in, void* out, void* stream) {
  if (N < 0 || N > 65534 || nfields < 1 || nfields > 65535)
    return fail(SHT_EINVAL, "need 0 <= N <= 65534 and 1 <= nfields <= 65535");
  if (!std::isfinite(scale)) return fail(SHT_EINVAL, "scale must be finite");
  // complex pairs: aligned to two elements
  const int al = dbl ? 16 : 8;
  int rc = check_ptr(in, "in", al);
  if (!rc) rc = check_ptr(out, "out", al);
  if (rc) return rc;
  return hip_check((hipError_t)launch_laplacian(N, nfields, scale, dbl != 0, in, out, stream), "laplacian launch");
}

int sht_grid_residual(long long n, long long n_per, int dbl, double alpha, const void* x, const void* kappa,
                      const void* y, const void* f, void* r, void* stream) {
  if (n < 1 || n_per < 1 || n % n_per) return fail(SHT_EINVAL, "need n >= 1 a multiple of n_per >= 1");
  if (!std::isfinite(alpha)) return fail(SHT_EINVAL, "alpha must be finite");
  const int al = dbl ? 8 : 4;  // element-aligned (16-byte vectors where all are)
  int rc = check_ptr(x, "x", al);
  if (!rc) rc = check_ptr(kappa, "kappa", al);
  if (!rc) rc = check_ptr(y, "y", al);
  if (!rc) rc = check_ptr(f, "f", al);
  if (!rc) rc = check_ptr(r, "r", al);
  if (rc) return rc;
  return hip_check((hipError_t)launch_residual(n, n_per, alpha, dbl != 0, x, kappa, y, f, r, stream),
                   "residual launch");
}

int sht_grid_inject(int J_fine, int I_fine, int J_coarse, int I_coarse, int nfields, int grid, int dbl,
                    const void* fine, void* coarse, void* stream) {
  if (nfields < 1 || nfields > 65535 || I_coarse < 1 || I_fine < I_coarse || I_fine % I_coarse)
    return fail(SHT_EINVAL, "need nfields >= 1 and I_fine a multiple of I_coarse");
  int rs = 0, r0 = 0;
  if (grid == SHT_GRID_CC_POLES) {
    if (J_coarse < 2 || J_fine < J_coarse || (J_fine - 1) % (J_coarse - 1))
      return fail(SHT_EINVAL, "CC grid with poles: need J_fine - 1 a multiple of J_coarse - 1 (J_coarse >= 2)");
    rs = (J_fine - 1) / (J_coarse - 1);
    r0 = 0;
  } else if (grid == SHT_GRID_FEJER2) {
    if (J_coarse < 1 || J_fine < J_coarse || (J_fine + 1) % (J_coarse + 1))
      return fail(SHT_EINVAL, "paper's grid: need J_fine + 1 a multiple of J_coarse + 1");
    rs = (J_fine + 1) / (J_coarse + 1);
    r0 = rs - 1;
  } else {
    return fail(SHT_EINVAL, "grid kind does not nest");
  }
  if (J_coarse > 65535) return fail(SHT_EINVAL, "J_coarse too large");
  const int al = dbl ? 8 : 4;  // element-aligned: scalar accesses
  int rc = check_ptr(fine, "fine", al);
  if (!rc) rc = check_ptr(coarse, "coarse", al);
  if (rc) return rc;
  if (fine == coarse) return fail(SHT_EINVAL, "fine and coarse must not overlap");
  return hip_check((hipError_t)launch_inject(J_fine, I_fine, J_coarse, I_coarse, nfields, rs, r0, I_fine / I_coarse,
                                             dbl != 0, fine, coarse, stream),
                   "inject launch");
}

sht_plan_t sht_plan(int N, int J, int I, int nfields) {
  sht_plan_t p = nullptr;
  if (build_plan(1, &N, &J, &I, &nfields, nullptr, &p) != SHT_OK) return nullptr;
  return p;
}

int sht_plan_ex(int N, int J, int I, int nfields, const sht_options* opts, sht_plan_t* out) {
  return build_plan(1, &N, &J, &I, &nfields, opts, out);
}

int sht_plan_multi(int nlevels, const int* N, const int* J, const int* I, const int* nfields,
                   const sht_options* opts, sht_plan_t* out) {
  return build_plan(nlevels, N, J, I, nfields, opts, out);
}

int sht_forward(sht_plan_t plan, const void* grid, void* spec, void* stream) {
  int rc;
  if ((rc = check_plan(plan)) || (rc = check_ptr(grid, "grid")) || (rc = check_ptr(spec, "spec"))) return rc;
  return run_dir(plan, DIR_FWD, grid, spec, stream);
}

int sht_forward_noalloc(sht_plan_t plan, const void* grid, void* spec, void* stream) {
  int rc;
  if ((rc = check_plan(plan)) || (rc = check_ptr(grid, "grid")) || (rc = check_ptr(spec, "spec"))) return rc;
  return run_forward_noalloc(plan, grid, spec, stream);
}

int sht_inverse(sht_plan_t plan, const void* spec, void* grid, void* stream) {
  int rc;
  if ((rc = check_plan(plan)) || (rc = check_ptr(spec, "spec")) || (rc = check_ptr(grid, "grid"))) return rc;
  return run_dir(plan, DIR_INV, spec, grid, stream);
}

int sht_forward_adjoint(sht_plan_t plan, const void* spec_bar, void* grid_bar, void* stream) {
  int rc;
  if ((rc = check_plan(plan)) || (rc = check_ptr(spec_bar, "spec_bar")) || (rc = check_ptr(grid_bar, "grid_bar")))
    return rc;
  return run_dir(plan, DIR_FWD_ADJ, spec_bar, grid_bar, stream);
}

int sht_inverse_adjoint(sht_plan_t plan, const void* grid_bar, void* spec_bar, void* stream) {
  int rc;
  if ((rc = check_plan(plan)) || (rc = check_ptr(grid_bar, "grid_bar")) || (rc = check_ptr(spec_bar, "spec_bar")))
    return rc;
  return run_dir(plan, DIR_INV_ADJ, grid_bar, spec_bar, stream);
}

int sht_plan_query(sht_plan_t plan, int key, void* out) {
  int rc;
  if ((rc = check_plan(plan))) return rc;
  if (!out) return fail(SHT_EINVAL, "out must not be NULL");
  const sht_plan_s* P = plan;
  switch (key) {
    case SHT_Q_NLEVELS: *(int*)out = P->nlev; return SHT_OK;
    case SHT_Q_NCOEF: *(int*)out = (P->lev[0].N + 1) * (P->lev[0].N + 2) / 2; return SHT_OK;
    case SHT_Q_EXACT: *(int*)out = P->exact ? 1 : 0; return SHT_OK;
    case SHT_Q_WORKSPACE_BYTES: *(size_t*)out = P->ws_bytes; return SHT_OK;
    case SHT_Q_TABLE_BYTES: *(size_t*)out = P->table_bytes; return SHT_OK;
    case SHT_Q_GRID_ELEMS: *(size_t*)out = P->grid_elems; return SHT_OK;
    case SHT_Q_SPEC_ELEMS: *(size_t*)out = P->spec_elems; return SHT_OK;
    case SHT_Q_FORM: *(int*)out = P->form; return SHT_OK;
    case SHT_Q_GRID_KIND: *(int*)out = P->grid; return SHT_OK;
    case SHT_Q_LEGENDRE_FLOPS: *(double*)out = P->flops; return SHT_OK;
    case SHT_Q_LEGENDRE_FLOPS_KEPT: *(double*)out = P->flops_kept; return SHT_OK;
    case SHT_Q_ZONAL_ONE_LAUNCH:
      *(int*)out = P->nlev > 1 ? (P->one_fwd ? 1 : 0) | (P->one_inv ? 2 : 0) : 0;
      return SHT_OK;
    default: break;
  }
  if (key >= SHT_Q_GRID_OFFSET && key < SHT_Q_GRID_OFFSET + P->nlev) {
    *(size_t*)out = (size_t)P->lev[key - SHT_Q_GRID_OFFSET].grid_off;
    return SHT_OK;
  }
  if (key >= SHT_Q_SPEC_OFFSET && key < SHT_Q_SPEC_OFFSET + P->nlev) {
    *(size_t*)out = (size_t)P->lev[key - SHT_Q_SPEC_OFFSET].spec_off;
    return SHT_OK;
  }
  return fail(SHT_EINVAL, "unknown query key");
}

int sht_host_tables(int N, int J, int grid, double* mu, double* w, double* alf) {
  if (N < 0) return fail(SHT_EINVAL, "N must be >= 0");
  if (!grid_args_ok(J, grid)) return fail(SHT_EINVAL, "bad J or grid kind");
  std::vector<double> m_(J), s_(J), w_(J);
  grid_nodes(J, grid, m_.data(), s_.data());
  grid_weights(J, grid, w_.data());
  if (mu) std::memcpy(mu, m_.data(), J * sizeof(double));
  if (w) std::memcpy(w, w_.data(), J * sizeof(double));
  if (alf) {
    int nth = (int)std::thread::hardware_concurrency();
    alf_table(N, (J + 1) / 2, m_.data(), s_.data(), alf, std::max(1, std::min(nth, 64)));
  }
  return SHT_OK;
}

int sht_plan_tables(sht_plan_t plan, double* mu, double* w, double* alf) {
  int rc;
  if ((rc = check_plan(plan))) return rc;
  return sht_host_tables(plan->lev[0].N, plan->lev[0].J, plan->grid, mu, w, alf);
}

int sht_plan_profile(sht_plan_t plan, int enable) {
  int rc;
  if ((rc = check_plan(plan))) return rc;
  plan->profile = enable ? 1 : 0;
  plan->ev_used = 0;
  plan->ev_stage.clear();
  return SHT_OK;
}

int sht_plan_profile_read(sht_plan_t plan, double* ms, int* counts) {
  int rc;
  if ((rc = check_plan(plan))) return rc;
  if (!ms || !counts) return fail(SHT_EINVAL, "ms and counts must not be NULL");
  for (int k = 0; k < ST_COUNT; ++k) {
    ms[k] = 0.0;
    counts[k] = 0;
  }
  if (plan->ev_used) {
    rc = hip_check(hipEventSynchronize(plan->ev_pool[plan->ev_used - 1]), "profile synchronize");
    if (rc) return rc;
  }
  for (size_t k = 0; k < plan->ev_stage.size() && 2 * k + 1 < plan->ev_used; ++k) {
    float t = 0.f;
    rc = hip_check(hipEventElapsedTime(&t, plan->ev_pool[2 * k], plan->ev_pool[2 * k + 1]), "profile read");
    if (rc) return rc;
    ms[plan->ev_stage[k]] += t;
    counts[plan->ev_stage[k]] += 1;
  }
  plan->ev_used = 0;
  plan->ev_stage.clear();
  return SHT_OK;
}

int sht_plan_destroy(sht_plan_t plan) {
  int rc;
  if ((rc = check_plan(plan))) return rc;
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.erase(plan);
  }
  plan->magic = 0;
  free_plan(plan);
  delete plan;
  return SHT_OK;
}

}  // extern "C"
