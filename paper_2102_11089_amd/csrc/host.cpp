// Host runtime behind include/ldpcci.h: argument validation, code upload, LDS layout and
// kernel selection.  Every step of decoding runs in the HIP kernels; this file only prepares
// their parameters and launches them on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ldpcci.h"
#include "kernels.hpp"

using namespace ldpc;

struct ldpc_code {
  int device;
  int M, N, E;
  int max_dv, max_dc, min_dc, max_touch, n_layers, max_layer_edges;
  uint64_t sig;  // hash of H (tuning key)
  std::vector<int> h_row_ptr, h_col, h_layer_ptr;
  std::vector<int> h_qc;  // quasi-cyclic base tables (empty for a plain CSR code)
  int nbr_max_cnt;
  int qc_Z, qc_mb, qc_nb, qc_nblk;
  int* d_buf;       // one device allocation holding every index array
  int* d_lut;       // 7 p0 tables (frac_bits 0..6), 257 entries each
  DevCode dev;
  DevCode* d_self;  // device copy of dev (batched launches)
  std::mutex rank_mu;  // guards gf2_rank, computed on the first ldpc_code_rank call
  int gf2_rank = -1;
};

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return LDPC_EHIP;
}

// Fault injection for tests of the error paths: LDPCCI_FAULT=alloc fails every scratch allocation
// as out of memory, LDPCCI_FAULT=launch fails every decode launch; nothing reaches the device.
enum { FAULT_NONE = 0, FAULT_ALLOC, FAULT_LAUNCH };
int injected_fault() {
  const char* v = std::getenv("LDPCCI_FAULT");
  if (!v) return FAULT_NONE;
  if (!std::strcmp(v, "alloc")) return FAULT_ALLOC;
  if (!std::strcmp(v, "launch")) return FAULT_LAUNCH;
  return FAULT_NONE;
}

// The process's abort flag: one int of fine-grained pinned host memory, mapped for every device,
// created with the first code handle (or the first ldpc_request_abort) and kept until the process
// ends.  Kernels read it before each frame they start.
std::mutex g_abort_mu;
int* g_abort_host = nullptr;
const int* g_abort_dev = nullptr;

int ensure_abort_flag() {
  std::lock_guard<std::mutex> lk(g_abort_mu);
  if (g_abort_host) return LDPC_OK;
  int* p = nullptr;
  hipError_t he = hipHostMalloc((void**)&p, sizeof(int), hipHostMallocMapped | hipHostMallocCoherent | hipHostMallocPortable);
  if (he != hipSuccess) return hip_fail(he);
  __atomic_store_n(p, 0, __ATOMIC_SEQ_CST);
  void* d = nullptr;
  he = hipHostGetDevicePointer(&d, p, 0);
  if (he != hipSuccess) {
    (void)hipHostFree(p);
    return hip_fail(he);
  }
  g_abort_dev = static_cast<const int*>(d);
  g_abort_host = p;
  return LDPC_OK;
}

int align16(int x) { return (x + 15) & ~15; }

// A kernel family's dynamic-LDS limit is raised with one hipFuncSetAttribute per variant (140 for
// the single-edge family), which costs more host time than a small decode: it is done once per
// device and family, and again only for a larger limit.
enum LdsFamily { FAM_BASELINE = 0, FAM_DYNAMIC, FAM_ME, FAM_BATCH, FAM_UNROLL };
hipError_t raise_lds_limit(int family, int bytes, hipError_t (*set)(int)) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, int> raised;  // (device, family) -> limit applied
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set(bytes);
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(dev, family);
  auto it = raised.find(key);
  if (it != raised.end() && it->second >= bytes) return hipSuccess;
  const hipError_t e = set(bytes);
  if (e == hipSuccess) raised[key] = bytes;
  return e;
}

// Stream-ordered scratch memory.  It comes from a pool of the library's own per device that keeps
// up to kPoolKeepBytes of freed memory for the next call: the device's default pool hands freed
// memory back to the system at every synchronization, so a caller that decodes, synchronizes and
// decodes again would map its scratch anew each time (measured: 35 us of a 1.27 ms adjoint call).
// The pools live until the process ends.  If a pool cannot be made, the default pool is used.
constexpr uint64_t kPoolKeepBytes = 2ull << 30;

hipMemPool_t scratch_pool(int dev) {
  static std::mutex mu;
  static std::map<int, hipMemPool_t> pools;  // device -> pool (nullptr: creation failed)
  std::lock_guard<std::mutex> lk(mu);
  auto it = pools.find(dev);
  if (it != pools.end()) return it->second;
  hipMemPoolProps props;
  std::memset(&props, 0, sizeof props);
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  hipMemPool_t pool = nullptr;
  if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
    (void)hipGetLastError();
    pool = nullptr;
  } else {
    uint64_t keep = kPoolKeepBytes;
    if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) (void)hipGetLastError();
  }
  pools[dev] = pool;
  return pool;
}

hipError_t scratch_alloc(void** p, size_t bytes, hipStream_t st) {
  if (injected_fault() == FAULT_ALLOC) return hipErrorOutOfMemory;
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return he;
  hipMemPool_t pool = scratch_pool(dev);
  return pool ? hipMallocFromPoolAsync(p, bytes, pool, st) : hipMallocAsync(p, bytes, st);
}

int device_lds_limit(int dev) {
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || v <= 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 65536;
  }
  return v;
}

int device_cu_count(int dev) {
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
  return v;
}

// architecture name and CU count: the key under which tuning results are stored
std::string device_tag(int dev) {
  hipDeviceProp_t p{};
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
    arch = p.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
  }
  return arch + "/" + std::to_string(device_cu_count(dev));
}

// FNV-1a over the parity-check matrix: equal codes share tuning entries
uint64_t code_signature(int M, int N, const int* row_ptr, const int* col, int E) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint32_t v) {
    for (int b = 0; b < 4; ++b) {
      h ^= (v >> (8 * b)) & 0xFFu;
      h *= 1099511628211ull;
    }
  };
  mix((uint32_t)M);
  mix((uint32_t)N);
  for (int m = 0; m <= M; ++m) mix((uint32_t)row_ptr[m]);
  for (int e = 0; e < E; ++e) mix((uint32_t)col[e]);
  return h;
}

double round_half_away(double x) { return x < 0 ? -std::floor(-x + 0.5) : std::floor(x + 0.5); }

// LDS layout of the single-edge / multi-edge dynamic decoders
struct DynLayout {
  int off_c2v, off_pre, off_L, off_Lt, off_D, off_ckey, off_dblk, off_cblk, off_dmask, off_cmask, off_syn;
  int off_v, off_grp, off_lut, off_topo, total;
  int nbd, nbc, nbd_words, nbc_words;
  int frame_base, frame_stride, wpb;  // shared region, then wpb frame regions of frame_stride bytes
};

// LDS bytes of a topology variant
long long topo_bytes(const ldpc_code* c, int topo) {
  if (topo == TOPO_QC) return c->h_qc.empty() ? -1 : (long long)c->h_qc.size() * 4;
  if (topo == TOPO_LDS) {
    const long long ints = (c->M + 1) + (c->N + 1) + 4LL * c->E;
    return 4LL * (ints + (ints & 1)) + 8LL * c->N;
  }
  return 0;
}

struct Dims {
  int E, N, M;
  long long topo_bytes;
  int nbr_passes;  // largest two-hop table of a VN, in passes of 64 lanes
};

// LDS of the single-edge kernels for wpb frames per workgroup: a shared region (p0 table in fixed
// point, topology tables) followed by wpb frame regions.  Frame arrays by storage mode: STORE_LDS
// c2v, pre, Lt, L, D; STORE_PRE_GLOBAL c2v, Lt, L, D; STORE_ALL_GLOBAL Lt, L, D; STORE_ALL_GLOBAL_LT
// L, D; STORE_FRAME_GLOBAL and STORE_FRAME_REC none of them; always the check keys, block maxima, dirty masks,
// syndrome bits and the two-hop staging.  Frame offsets are relative to the frame's region.
DynLayout dyn_layout_dims(const Dims& c, bool fixed, int store, int wpb) {
  DynLayout L{};
  const int msg = fixed ? 1 : 4, llr = 4;
  L.nbd = (c.N + WAVE - 1) / WAVE;
  L.nbc = (c.M + WAVE - 1) / WAVE;
  L.nbd_words = (L.nbd + 31) / 32;
  L.nbc_words = (L.nbc + 31) / 32;
  int o = 0;
  L.off_lut = o; if (fixed) o = align16(o + 257 * 4);
  L.off_topo = o; o = align16(o + (int)std::max(0LL, c.topo_bytes));
  L.frame_base = o;
  int f = 0;
  L.off_c2v = f; if (store < STORE_ALL_GLOBAL) f = align16(f + c.E * msg);
  L.off_pre = f; if (store == STORE_LDS) f = align16(f + c.E * msg);
  const bool frame = store == STORE_FRAME_GLOBAL || store == STORE_FRAME_REC || store == STORE_FRAME_ALL;
  L.off_L = f; if (!frame) f = align16(f + c.N * llr);
  L.off_Lt = f; if (store < STORE_ALL_GLOBAL_LT) f = align16(f + c.N * llr);
  L.off_D = f; if (!frame) f = align16(f + c.N * 4);
  const bool keys_global = store == STORE_FRAME_ALL;
  L.off_ckey = f; if (!keys_global) f = align16(f + c.M * 4);
  L.off_dblk = f; f = align16(f + L.nbd * 8);
  L.off_cblk = f; f = align16(f + L.nbc * 8);
  L.off_dmask = f; f = align16(f + L.nbd_words * 4);
  L.off_cmask = f; f = align16(f + L.nbc_words * 4);
  L.off_syn = f; f = align16(f + ((c.M + 31) / 32) * 4);
  // late-CI VN per table lane (in the global slot when the frame has one)
  L.off_v = f; if (store < STORE_ALL_GLOBAL) f = align16(f + std::max(1, std::min(c.nbr_passes, NBR_PMAX)) * WAVE * 4);
  L.off_grp = f; f = align16(f + kGroupBytes);  // sums for VNs met twice in a two-hop table
  L.frame_stride = f;
  L.wpb = wpb;
  L.total = L.frame_base + wpb * f;
  return L;
}

DynLayout dyn_layout(const ldpc_code* c, bool fixed, int store, int topo, int wpb) {
  return dyn_layout_dims(Dims{c->E, c->N, c->M, topo_bytes(c, topo), (c->nbr_max_cnt + WAVE - 1) / WAVE}, fixed,
                         store, wpb);
}


// LDS layout of the multi-edge decoder; returns the total bytes
struct MeLayout {
  int off_c2v, off_pre, off_L, off_Lt, off_D, off_hist, off_synw, off_rowmark, off_vnmark, off_rows, off_sel;
  int off_cand, off_misc, off_lut, off_topo, off_rows2, off_vnmulti, off_mpref, off_macc, total, rows_cap, cand_cap;
};

// LDS of the unrolled kernels: forward (c2v, L); backward adds the adjoints and the segment tape
// (the weight gradients accumulate in the frame's global scratch row)
void unroll_layout(const ldpc_code* c, int K, UnrollParams& U) {
  int o = 0;
  U.off_c2v = o; o = align16(o + c->E * 4);
  U.off_L = o; o = align16(o + c->N * 4);
  U.lds_fwd = o;
  U.off_ch = o; o = align16(o + c->E * 4);
  U.off_Lh = o; o = align16(o + c->N * 4);
  U.tstride = c->max_dc;  // tape row: the inputs of one check
  U.off_tape = o; o = align16(o + K * U.tstride * 8);
  U.off_tape_hdr = o; o = align16(o + K * 16);  // (p, c_old, dw) per step
  U.lds_bwd = o;
}

MeLayout me_layout(const ldpc_code* c, bool fixed, bool msg_global, int topo, int n_p, int n_g, int fill) {
  MeLayout L{};
  const int msg = fixed ? 1 : 4;
  const int nsw = (c->M + 31) / 32, nvw = (c->N + 31) / 32;
  L.rows_cap = n_p * c->max_dv;
  L.cand_cap = fill == LDPC_FILL_HASH ? 512 : 0;
  int o = 0;
  L.off_c2v = L.off_pre = o; if (!msg_global) o = align16(o + 2 * c->E * msg);  // (c2v, pre) pairs
  L.off_L = o; o = align16(o + c->N * 4);
  L.off_Lt = o; o = align16(o + c->N * 4);
  L.off_D = o; o = align16(o + c->N * 4);
  L.off_hist = o; o = align16(o + n_g * 4);
  L.off_synw = o; o = align16(o + nsw * 4);
  L.off_rowmark = o; o = align16(o + nsw * 4);
  L.off_vnmark = o; o = align16(o + nvw * 4);
  L.off_vnmulti = o; o = align16(o + nvw * 4);  // VNs that two or more checks of a step change
  L.off_mpref = o; if (!fixed) o = align16(o + nvw * 4);             // their rank: prefix counts per word
  L.off_macc = o; if (!fixed) o = align16(o + kMeAccSlots * 8);      // and their exact 64-bit sums
  L.off_rows = o; o = align16(o + L.rows_cap * 4);
  L.off_rows2 = o; o = align16(o + L.rows_cap * 4);  // the same checks sorted by block size
  L.off_sel = o; o = align16(o + 5 * 64 * 4);  // set, sorted set, class counters, P', m* per VN
  L.off_cand = o; o = align16(o + L.cand_cap * 12);
  L.off_misc = o; o = align16(o + 48 * 4);  // 32 counters, one word per wavefront
  L.off_lut = o; if (fixed) o = align16(o + 257 * 4);
  L.off_topo = o; o = align16(o + (int)std::max(0LL, topo_bytes(c, topo)));
  L.total = o;
  return L;
}

}  // namespace

extern "C" {

const char* ldpc_strerror(int code) {
  switch (code) {
    case LDPC_OK: return "ok";
    case LDPC_EINVAL: return "invalid argument";
    case LDPC_ENOMEM: return "out of memory";
    case LDPC_EHIP: return "HIP runtime error";
    case LDPC_ECAPACITY: return "frame state exceeds on-chip memory";
    case LDPC_EUNSUPPORTED: return "unsupported schedule, arithmetic or code shape";
    default: return "unknown error";
  }
}

int ldpc_last_hip_error(void) { return g_last_hip; }

int ldpc_request_abort(int32_t on) {
  if (int rc = ensure_abort_flag()) return rc;
  __atomic_store_n(g_abort_host, on ? 1 : 0, __ATOMIC_SEQ_CST);
  return LDPC_OK;
}

static int create_code(int32_t M, int32_t N, const int32_t* row_ptr, const int32_t* col_idx,
                       const int32_t* layer_ptr, int32_t n_layers, const std::vector<int>* qc, int qZ, int qmb,
                       int qnb, int qnblk, ldpc_code** out) {
  if (!out) return LDPC_EINVAL;
  *out = nullptr;
  if (M <= 0 || N <= 0 || !row_ptr || !col_idx) return LDPC_EINVAL;
  if (N >= (1 << 24)) return LDPC_EUNSUPPORTED;  // VN indices share a word with 8 flag bits in the two-hop table
  if (row_ptr[0] != 0) return LDPC_EINVAL;
  for (int m = 0; m < M; ++m)
    if (row_ptr[m + 1] - row_ptr[m] < 2) return LDPC_EINVAL;
  const long long E64 = row_ptr[M];
  if (E64 <= 0 || E64 > (1 << 28)) return LDPC_EINVAL;
  const int E = (int)E64;
  std::vector<int> vdeg(N, 0);
  for (int m = 0; m < M; ++m) {
    for (int e = row_ptr[m]; e < row_ptr[m + 1]; ++e) {
      int n = col_idx[e];
      if (n < 0 || n >= N) return LDPC_EINVAL;
      if (e > row_ptr[m] && col_idx[e - 1] >= n) return LDPC_EINVAL;
      vdeg[n] += 1;
    }
  }
  for (int n = 0; n < N; ++n)
    if (vdeg[n] < 1) return LDPC_EINVAL;
  std::vector<int> lp;
  if (layer_ptr) {
    if (n_layers < 1 || layer_ptr[0] != 0 || layer_ptr[n_layers] != M) return LDPC_EINVAL;
    std::vector<int> mark(N, -1);
    for (int l = 0; l < n_layers; ++l) {
      if (layer_ptr[l + 1] <= layer_ptr[l]) return LDPC_EINVAL;
      for (int e = row_ptr[layer_ptr[l]]; e < row_ptr[layer_ptr[l + 1]]; ++e) {
        if (mark[col_idx[e]] == l) return LDPC_EINVAL;  // two rows of one layer share a VN
        mark[col_idx[e]] = l;
      }
    }
    lp.assign(layer_ptr, layer_ptr + n_layers + 1);
  } else {
    lp.resize(M + 1);
    for (int m = 0; m <= M; ++m) lp[m] = m;
  }
  ldpc_code* c = new (std::nothrow) ldpc_code();
  if (!c) return LDPC_ENOMEM;
  c->M = M;
  c->N = N;
  c->E = E;
  c->n_layers = (int)lp.size() - 1;
  c->h_row_ptr.assign(row_ptr, row_ptr + M + 1);
  c->sig = code_signature(M, N, row_ptr, col_idx, E);
  c->h_col.assign(col_idx, col_idx + E);
  c->h_layer_ptr = lp;
  // derived host arrays: row of edge, CSC (checks ascending inside a column)
  std::vector<int> row_of(E), col_ptr(N + 1, 0), col_row(E), col_eid(E);
  for (int m = 0; m < M; ++m)
    for (int e = row_ptr[m]; e < row_ptr[m + 1]; ++e) row_of[e] = m;
  for (int n = 0; n < N; ++n) col_ptr[n + 1] = col_ptr[n] + vdeg[n];
  std::vector<int> fill(col_ptr.begin(), col_ptr.end() - 1);
  for (int e = 0; e < E; ++e) {  // row-major traversal keeps checks ascending per column
    int n = col_idx[e];
    col_row[fill[n]] = row_of[e];
    col_eid[fill[n]] = e;
    fill[n] += 1;
  }
  c->max_dv = *std::max_element(vdeg.begin(), vdeg.end());
  c->max_dc = 0;
  c->min_dc = M > 0 ? row_ptr[1] - row_ptr[0] : 0;
  for (int m = 0; m < M; ++m) {
    c->max_dc = std::max(c->max_dc, row_ptr[m + 1] - row_ptr[m]);
    c->min_dc = std::min(c->min_dc, row_ptr[m + 1] - row_ptr[m]);
  }
  c->max_touch = 0;
  for (int n = 0; n < N; ++n) {
    int s = 0;
    for (int k = col_ptr[n]; k < col_ptr[n + 1]; ++k) s += row_ptr[col_row[k] + 1] - row_ptr[col_row[k]];
    c->max_touch = std::max(c->max_touch, s);
  }
  c->max_layer_edges = 0;
  for (int l = 0; l < c->n_layers; ++l)
    c->max_layer_edges = std::max(c->max_layer_edges, row_ptr[lp[l + 1]] - row_ptr[lp[l]]);
  // two-hop neighbourhood table: per VN, every check of the VN as an aligned power-of-two block
  // of lanes (largest first, so every block starts at a multiple of its size), in VN order
  std::vector<int> nbr, nbr_idx(2 * (size_t)N), seen(N, 0), group(N, -1);
  int next_group = 0;
  c->nbr_max_cnt = 0;
  for (int n = 0; n < N; ++n) {
    std::vector<std::pair<int, int>> blocks;  // (log2 size, check)
    for (int k = col_ptr[n]; k < col_ptr[n + 1]; ++k) {
      const int m = col_row[k], dc = row_ptr[m + 1] - row_ptr[m];
      int l2 = 0;
      while ((1 << l2) < dc) ++l2;
      blocks.push_back({l2, m});
    }
    std::stable_sort(blocks.begin(), blocks.end(), [](auto& a, auto& b) { return a.first > b.first; });
    const int off = (int)(nbr.size() / 2);
    // VNs other than n met in more than one check of n (4-cycles through n): flagged, because the
    // kernels then sum several changes into their Lt
    for (auto& bk : blocks)
      for (int x = row_ptr[bk.second]; x < row_ptr[bk.second + 1]; ++x) seen[col_idx[x]] += 1;
    for (auto& bk : blocks) {
      const int l2 = bk.first, m = bk.second, rs = row_ptr[m], dc = row_ptr[m + 1] - rs;
      if (l2 > 5) {
        delete c;
        return LDPC_EUNSUPPORTED;  // a check of degree > 32
      }
      for (int p = 0; p < (1 << l2); ++p) {
        const bool valid = p < dc;
        const int j = valid ? col_idx[rs + p] : 0;
        const bool twice = valid && j != n && seen[j] > 1;
        int g = 0;
        if (twice) {  // group id of the VN: first-seen order, the last id shared by any further VNs
          if (group[j] < 0) group[j] = std::min(next_group++, kGroups);
          g = group[j];
        }
        nbr.push_back(valid ? rs + p : -1);
        nbr.push_back(j | (l2 << 24) | ((p == 0 ? 1 : 0) << 27) | ((twice ? 1 : 0) << 28) | (g << 29));
      }
    }
    for (auto& bk : blocks)
      for (int x = row_ptr[bk.second]; x < row_ptr[bk.second + 1]; ++x) {
        seen[col_idx[x]] = 0;
        group[col_idx[x]] = -1;
      }
    next_group = 0;
    const int cnt = (int)(nbr.size() / 2) - off;
    nbr_idx[2 * n] = off;
    nbr_idx[2 * n + 1] = cnt;
    c->nbr_max_cnt = std::max(c->nbr_max_cnt, cnt);
  }
  // one device buffer: row_ptr, col, row_of, col_ptr, col_row, col_eid, layer_ptr, 7 LUTs
  std::vector<int> blob;
  auto put = [&](const std::vector<int>& v) {
    size_t o = blob.size();
    blob.insert(blob.end(), v.begin(), v.end());
    while (blob.size() % 4) blob.push_back(0);
    return o;
  };
  size_t o_rp = put(c->h_row_ptr), o_col = put(c->h_col), o_ro = put(row_of), o_cp = put(col_ptr);
  size_t o_cr = put(col_row), o_ce = put(col_eid), o_lp = put(lp);
  std::vector<int> luts(7 * 257);
  for (int f = 0; f <= 6; ++f)
    for (int x = -128; x <= 128; ++x)
      luts[f * 257 + x + 128] = (int)round_half_away(32767.0 * std::tanh(0.5 * std::ldexp((double)x, -f)));
  size_t o_lut = put(luts);
  size_t o_nbr = put(nbr), o_nidx = put(nbr_idx);
  size_t o_qc = 0;
  if (qc) {
    // per base column: (offset of the column's first VN, entries per VN); VNs of one column
    // have equal check degrees, so off(j Z + c) = off(j Z) + c cnt
    std::vector<int> q2 = *qc;
    for (int j = 0; j < qnb; ++j) {
      q2.push_back(nbr_idx[2 * ((size_t)j * qZ)]);
      q2.push_back(nbr_idx[2 * ((size_t)j * qZ) + 1]);
    }
    for (int i = 0; i < qmb; ++i) {  // FastDiv of each base-row degree
      const FastDiv f = FastDiv::of((uint32_t)(*qc)[i]);
      q2.push_back((int)f.mul);
      q2.push_back((int)f.sh);
    }
    // base rows by descending degree (lower index first on ties): the order in which flooding's
    // wavefronts take rows, so that the longest rows start first
    std::vector<int> order(qmb);
    for (int i = 0; i < qmb; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return (*qc)[a] > (*qc)[b]; });
    q2.insert(q2.end(), order.begin(), order.end());
    c->h_qc = q2;
    c->qc_Z = qZ;
    c->qc_mb = qmb;
    c->qc_nb = qnb;
    c->qc_nblk = qnblk;
    o_qc = put(c->h_qc);
  }
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return LDPC_EHIP;
  }
  if (int rc = ensure_abort_flag()) {
    delete c;
    return rc;
  }
  hipError_t he = hipMalloc((void**)&c->d_buf, blob.size() * sizeof(int));
  if (he != hipSuccess) {
    delete c;
    g_last_hip = (int)he;
    return he == hipErrorOutOfMemory ? LDPC_ENOMEM : LDPC_EHIP;
  }
  he = hipMemcpy(c->d_buf, blob.data(), blob.size() * sizeof(int), hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    (void)hipFree(c->d_buf);
    delete c;
    return hip_fail(he);
  }
  DevCode& d = c->dev;
  d.M = M;
  d.N = N;
  d.E = E;
  d.max_dc = c->max_dc;
  d.max_dv = c->max_dv;
  d.max_touch = c->max_touch;
  d.n_layers = c->n_layers;
  d.row_ptr = c->d_buf + o_rp;
  d.col = c->d_buf + o_col;
  d.row_of = c->d_buf + o_ro;
  d.col_ptr = c->d_buf + o_cp;
  d.col_row = c->d_buf + o_cr;
  d.col_eid = c->d_buf + o_ce;
  d.layer_ptr = c->d_buf + o_lp;
  c->d_lut = c->d_buf + o_lut;
  d.nbr = reinterpret_cast<const int2*>(c->d_buf + o_nbr);
  d.nbr_idx = reinterpret_cast<const int2*>(c->d_buf + o_nidx);
  d.nbr_col = nullptr;
  d.nbr_max_cnt = c->nbr_max_cnt;
  d.qc = DevQC{};
  if (qc) {
    // table order: bdeg[mb], bptr[mb+1], brow[2 nblk], bcol_ptr[nb+1], bcol[4 nblk], rowmap[nblk]
    const int* q0 = c->d_buf + o_qc;
    d.qc.Z = qZ;
    d.qc.mb = qmb;
    d.qc.nb = qnb;
    d.qc.nblk = qnblk;
    d.qc.bdeg = q0;
    d.qc.bptr = q0 + qmb;
    d.qc.brow = d.qc.bptr + (qmb + 1);
    d.qc.bcol_ptr = d.qc.brow + 2 * qnblk;
    d.qc.bcol = d.qc.bcol_ptr + (qnb + 1);
    d.qc.rowmap = d.qc.bcol + 4 * qnblk;
    d.qc.words = (int)c->h_qc.size();
    d.nbr_col = reinterpret_cast<const int2*>(d.qc.rowmap + qnblk);
    d.qc.bdiv = d.qc.rowmap + qnblk + 2 * qnb;
    d.qc.border = d.qc.bdiv + 2 * qmb;
    d.qc.zdiv = FastDiv::of((uint32_t)qZ);
  }
  he = hipMalloc((void**)&c->d_self, sizeof(DevCode));
  if (he == hipSuccess) he = hipMemcpy(c->d_self, &c->dev, sizeof(DevCode), hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    if (c->d_self) (void)hipFree(c->d_self);
    (void)hipFree(c->d_buf);
    delete c;
    return hip_fail(he);
  }
  *out = c;
  return LDPC_OK;
}

int ldpc_code_from_csr(int32_t M, int32_t N, const int32_t* row_ptr, const int32_t* col_idx,
                       const int32_t* layer_ptr, int32_t n_layers, ldpc_code** out) {
  return create_code(M, N, row_ptr, col_idx, layer_ptr, n_layers, nullptr, 0, 0, 0, 0, out);
}

int ldpc_code_from_qc(int32_t mb, int32_t nb, int32_t Z, const int32_t* shift, ldpc_code** out) {
  if (!out) return LDPC_EINVAL;
  *out = nullptr;
  if (mb <= 0 || nb <= 0 || Z <= 0 || !shift) return LDPC_EINVAL;
  if ((long long)nb * Z > (1 << 26) || (long long)mb * Z > (1 << 26)) return LDPC_EINVAL;
  std::vector<int> bdeg(mb, 0), bptr(mb + 1, 0), brow, bcol_ptr(nb + 1, 0), bcol, rowmap;
  for (int i = 0; i < mb; ++i) {
    for (int j = 0; j < nb; ++j) {
      const int sh = shift[(size_t)i * nb + j];
      if (sh < -1 || sh >= Z) return LDPC_EINVAL;
      if (sh >= 0) {
        brow.push_back(j);
        brow.push_back(sh);
        rowmap.push_back(i);
        bdeg[i] += 1;
        bcol_ptr[j + 1] += 1;
      }
    }
    if (bdeg[i] < 2) return LDPC_EINVAL;
    bptr[i + 1] = bptr[i] + bdeg[i];
  }
  const int nblk = bptr[mb];
  for (int j = 0; j < nb; ++j) {
    if (bcol_ptr[j + 1] < 1) return LDPC_EINVAL;
    bcol_ptr[j + 1] += bcol_ptr[j];
  }
  bcol.assign(4 * (size_t)nblk, 0);
  std::vector<int> fillc(bcol_ptr.begin(), bcol_ptr.end() - 1);
  for (int i = 0; i < mb; ++i) {
    for (int k = 0; k < bdeg[i]; ++k) {  // ascending i per column by construction
      const int j = brow[2 * (bptr[i] + k)], sh = brow[2 * (bptr[i] + k) + 1];
      const int x = fillc[j]++;
      bcol[4 * x] = i;
      bcol[4 * x + 1] = sh;
      bcol[4 * x + 2] = k;
    }
  }
  std::vector<int> qc;
  qc.insert(qc.end(), bdeg.begin(), bdeg.end());
  qc.insert(qc.end(), bptr.begin(), bptr.end());
  qc.insert(qc.end(), brow.begin(), brow.end());
  qc.insert(qc.end(), bcol_ptr.begin(), bcol_ptr.end());
  qc.insert(qc.end(), bcol.begin(), bcol.end());
  qc.insert(qc.end(), rowmap.begin(), rowmap.end());
  // expanded CSR: check i Z + r meets VN j Z + ((r + shift) mod Z), VNs ascending (j ascending)
  const int M = mb * Z, N = nb * Z;
  std::vector<int> row_ptr(M + 1, 0), col((size_t)nblk * Z), layer(mb + 1);
  for (int i = 0; i < mb; ++i) {
    layer[i] = i * Z;
    for (int r = 0; r < Z; ++r) {
      const int m = i * Z + r;
      row_ptr[m + 1] = row_ptr[m] + bdeg[i];
      for (int k = 0; k < bdeg[i]; ++k) {
        const int j = brow[2 * (bptr[i] + k)], sh = brow[2 * (bptr[i] + k) + 1];
        col[row_ptr[m] + k] = j * Z + (r + sh) % Z;
      }
    }
  }
  layer[mb] = M;
  return create_code(M, N, row_ptr.data(), col.data(), layer.data(), mb, &qc, Z, mb, nb, nblk, out);
}

int ldpc_code_info(const ldpc_code* c, ldpc_code_stats* out) {
  if (!c || !out) return LDPC_EINVAL;
  out->M = c->M;
  out->N = c->N;
  out->E = c->E;
  out->max_dv = c->max_dv;
  out->max_dc = c->max_dc;
  out->n_layers = c->n_layers;
  out->max_touch = c->max_touch;
  out->mean_dv = (float)((double)c->E / c->N);
  out->mean_dc = (float)((double)c->E / c->M);
  {
    std::lock_guard<std::mutex> g(const_cast<ldpc_code*>(c)->rank_mu);
    out->gf2_rank = c->gf2_rank;
  }
  out->reserved = 0;
  const int topo = c->h_qc.empty() ? TOPO_LDS : TOPO_QC;
  out->lds_bytes_f32 = dyn_layout(c, false, STORE_LDS, topo, 1).total;
  out->lds_bytes_fix = dyn_layout(c, true, STORE_LDS, topo, 1).total;
  return LDPC_OK;
}

// Rank of H over GF(2) by Gaussian elimination on bit-packed rows: every row is reduced by the
// pivots found so far, in column order.  O(M^2 N / 64) word operations, M N / 8 bytes.
static int gf2_rank_of(const ldpc_code* c) {
  const int M = c->M, N = c->N, W = (N + 63) / 64;
  std::vector<uint64_t> A;
  try {
    A.assign((size_t)M * W, 0);
  } catch (const std::bad_alloc&) {
    return -1;
  }
  for (int m = 0; m < M; ++m)
    for (int e = c->h_row_ptr[m]; e < c->h_row_ptr[m + 1]; ++e) {
      const int n = c->h_col[e];
      A[(size_t)m * W + (n >> 6)] |= 1ull << (n & 63);
    }
  int rank = 0;
  for (int col = 0; col < N && rank < M; ++col) {
    const int w = col >> 6;
    const uint64_t bit = 1ull << (col & 63);
    int piv = -1;
    for (int m = rank; m < M; ++m)
      if (A[(size_t)m * W + w] & bit) {
        piv = m;
        break;
      }
    if (piv < 0) continue;
    if (piv != rank)
      std::swap_ranges(A.begin() + (size_t)piv * W, A.begin() + (size_t)(piv + 1) * W, A.begin() + (size_t)rank * W);
    const uint64_t* pr = &A[(size_t)rank * W];
    for (int m = piv + 1; m < M; ++m) {  // rows between rank and piv have no bit in this column
      uint64_t* r = &A[(size_t)m * W];
      if (r[w] & bit)
        for (int k = w; k < W; ++k) r[k] ^= pr[k];  // the pivot row has no bit before column col
    }
    rank += 1;
  }
  return rank;
}

int ldpc_code_rank(const ldpc_code* c, int32_t* rank) {
  if (!c || !rank) return LDPC_EINVAL;
  ldpc_code* cc = const_cast<ldpc_code*>(c);
  std::lock_guard<std::mutex> g(cc->rank_mu);
  if (cc->gf2_rank < 0) {
    const int r = gf2_rank_of(c);
    if (r < 0) return LDPC_ENOMEM;
    cc->gf2_rank = r;
  }
  *rank = cc->gf2_rank;
  return LDPC_OK;
}

void ldpc_code_free(ldpc_code* c) {
  if (!c) return;
  if (c->d_buf) (void)hipFree(c->d_buf);
  if (c->d_self) (void)hipFree(c->d_self);
  delete c;
}

}  // extern "C"

namespace {

// A decode call resolved to one kernel launch: parameters, launch shape and scratch size.
struct DecodePlan {
  int which = 0;  // 0 flooding/layered, 1 single-edge (RBP, CIRBP, replay), 2 ME-CIRBP
  bool fixed = false;
  BaseParams base{};
  DynParams dyn{};
  MeParams me{};
  int grid = 0, block = WAVE, topo = TOPO_GLOBAL;
  int store = STORE_LDS;      // single-edge: Store; ME: STORE_LDS or STORE_ALL_GLOBAL (c2v and pre in global)
  bool persistent = false;    // single-edge: persistent grid fed by a work queue at the front of scratch
  size_t scratch_bytes = 0;
  int lds_limit = 0;
};

bool valid_block(int b) { return b >= 64 && b <= 1024 && b % 64 == 0; }

constexpr size_t kQueueBytes = 256;  // work-queue counter at the front of a persistent launch's scratch

// global slot of one frame when its messages live in global memory, each part 256-byte aligned:
// (c2v, pre) pairs for E edges; Lt (messages + Lt), or Lt, L and D (split arrays), or one 8-byte
// (Lt, L) record per VN (record layouts); the M check keys (keys global); the late-CI staging
void all_global_slot(int E, int N, int M, int nbr_passes, bool fixed, int store, DynParams& P) {
  auto up = [](long long x) { return (x + 255) / 256 * 256; };
  long long o = up(2LL * E * (fixed ? 1 : 4));
  P.slot_lt_off = P.slot_l_off = P.slot_d_off = (int)o;
  P.slot_ckey_off = 0;
  if (store == STORE_FRAME_REC || store == STORE_FRAME_ALL) {
    o = up(o + 8LL * N);
  } else {
    if (store >= STORE_ALL_GLOBAL_LT) o = up(o + 4LL * N);
    if (store == STORE_FRAME_GLOBAL) {
      P.slot_l_off = (int)o;
      o = up(o + 4LL * N);
      P.slot_d_off = (int)o;
      o = up(o + 4LL * N);
    }
  }
  if (store == STORE_FRAME_ALL) {
    P.slot_ckey_off = (int)o;
    o = up(o + 4LL * M);
  }
  P.slot_tj_off = (int)o;
  P.slot_bytes = up(o + 4LL * WAVE * std::max(1, std::min(nbr_passes, NBR_PMAX)));
}

// tuning knob -> candidate topologies (empty: the knob does not apply to this code)
std::vector<int> topo_choices(const ldpc_code* c, int knob) {
  switch (knob) {
    case LDPC_TOPO_GLOBAL: return {TOPO_GLOBAL};
    case LDPC_TOPO_LDS: return {TOPO_LDS};
    case LDPC_TOPO_QC: return c->h_qc.empty() ? std::vector<int>{} : std::vector<int>{TOPO_QC};
    default:
      return c->h_qc.empty() ? std::vector<int>{TOPO_LDS, TOPO_GLOBAL} : std::vector<int>{TOPO_QC, TOPO_GLOBAL};
  }
}

int check_tuning(const ldpc_tuning* t) {
  if (!t) return LDPC_OK;
  if (t->block != 0 && !valid_block(t->block)) return LDPC_EINVAL;
  if (t->frames_per_cu < 0 || t->frames_per_cu > 32) return LDPC_EINVAL;
  if (t->storage < LDPC_STORE_AUTO || t->storage > LDPC_STORE_GLOBAL_STATE) return LDPC_EINVAL;
  if (t->topology < LDPC_TOPO_AUTO || t->topology > LDPC_TOPO_QC) return LDPC_EINVAL;
  return LDPC_OK;
}

// Validate a decode request and resolve it to a launch plan.  tune (nullable) overrides the
// default storage / topology / launch-shape policy.
// plan_only: shape the launch without the buffers (llr_in, out and replay may be null)
int plan_decode(const ldpc_code* c, const ldpc_schedule* s, const float* llr_in, int32_t B, int64_t max_updates,
                const int32_t* replay, int64_t replay_len, const ldpc_outputs* out, const ldpc_tuning* tune,
                DecodePlan& pl, bool plan_only = false) {
  const ldpc_outputs no_out{};
  if (plan_only && !out) out = &no_out;
  if (!c || !s || !out || B < 0 || max_updates < 0) return LDPC_EINVAL;
  if (!plan_only && B > 0 && (!llr_in || !out->bits || !out->updates_used)) return LDPC_EINVAL;
  if (s->kind < LDPC_FLOODING || s->kind > LDPC_ME_LMD_CIRBP) return LDPC_EINVAL;
  if (s->arith != LDPC_SPA_F32 && s->arith != LDPC_MS_FIX) return LDPC_EINVAL;
  const bool fixed = s->arith == LDPC_MS_FIX;
  if (fixed && (s->q_bits < 2 || s->q_bits > 8 || s->frac_bits < 0 || s->frac_bits > 6)) return LDPC_EINVAL;
  if (s->check_every < 0) return LDPC_EINVAL;
  if (!(s->gamma >= 0.0f) || !std::isfinite(s->gamma)) return LDPC_EINVAL;
  if (s->kind == LDPC_REPLAY && ((!plan_only && !replay) || replay_len < 0)) return LDPC_EINVAL;
  const bool me = s->kind == LDPC_ME_CIRBP || s->kind == LDPC_ME_LMD_CIRBP;
  if (me && (s->n_p < 1 || s->n_p > 64 || s->n_g < 1 || s->n_g > 65535 ||
                                   (s->fill != LDPC_FILL_LOWEST && s->fill != LDPC_FILL_HASH)))
    return LDPC_EINVAL;
  if (int rc = check_tuning(tune)) return rc;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LDPC_EHIP;
  if (dev != c->device) return LDPC_EINVAL;
  const ldpc_tuning none{};
  const ldpc_tuning& T = tune ? *tune : none;
  pl = DecodePlan{};
  pl.fixed = fixed;
  pl.lds_limit = std::min(device_lds_limit(dev), 160 * 1024);
  const int ncu = device_cu_count(dev);
  const int qmax = (1 << (std::max(s->q_bits, 2) - 1)) - 1;
  const float scale = std::ldexp(1.0f, fixed ? s->frac_bits : 0);

  DecOut o;
  o.bits = out->bits;
  o.llr_out = out->llr_out;
  o.updates_used = out->updates_used;
  o.steps_used = out->steps_used;
  o.fallbacks = out->fallbacks;
  o.trace = out->trace;
  o.dump_c2v = out->dump_c2v;
  o.dump_pre = out->dump_pre;
  o.dump_L = out->dump_L;
  o.dump_Lt = out->dump_Lt;
  o.dump_D = out->dump_D;
  o.abort = ldpc::abort_flag_address();

  if (s->kind == LDPC_FLOODING || s->kind == LDPC_LAYERED) {
    BaseParams& P = pl.base;
    P.kind = s->kind;
    P.B = B;
    P.max_updates = max_updates;
    P.check_every = s->check_every;
    P.llr = llr_in;
    P.out = o;
    P.qmax = qmax;
    P.scale = scale;
    P.c2v_global = nullptr;
    P.queue = nullptr;
    P.slot_edges = c->E;
    pl.which = 0;
    pl.store = STORE_LDS;
    const int msg = fixed ? 1 : 4;
    const int syn = ((c->M + 31) / 32) * 4;
    // topology: quasi-cyclic base tables, else CSR copies in LDS when they fit, else global arrays
    std::vector<int> tps = c->h_qc.empty() ? std::vector<int>{TOPO_LDS, TOPO_GLOBAL} : std::vector<int>{TOPO_QC};
    if (T.topology) {
      tps = topo_choices(c, T.topology);
      if (tps.empty()) return LDPC_EUNSUPPORTED;
    }
    if (s->kind == LDPC_FLOODING) {
      // one frame per workgroup, one workgroup per frame (the hardware hands out workgroups as
      // others finish): c2v, L, channel values, syndrome words, counter, topology copy
      bool found = false;
      for (int tp : tps) {
        int off = 0;
        P.off_c2v = off; off = align16(off + c->E * msg);
        P.off_L = off; off = align16(off + c->N * 4);
        P.off_ch = off; off = align16(off + c->N * 4);
        P.off_syn = off; off = align16(off + syn);
        P.off_misc = off; off = align16(off + 16);
        P.off_topo = off; off = align16(off + (int)topo_bytes(c, tp));
        P.lds_bytes = off;
        P.frame_base = 0;
        P.frame_stride = off;
        P.wpb = 1;
        if (off <= pl.lds_limit) {
          pl.topo = tp;
          found = true;
          break;
        }
      }
      if (!found) return LDPC_ECAPACITY;
      const int work = std::max(c->M, c->N);
      pl.block = T.block ? T.block : (work >= 2048 ? 1024 : (work >= 512 ? 256 : (work >= 128 ? 128 : 64)));
      pl.grid = B;
      return LDPC_OK;
    }
    // layered: one frame per wavefront; wpb frames per workgroup share the topology copy.  c2v in
    // LDS when that keeps at least as many frames per CU as c2v in a global slot would
    std::vector<bool> c2v_opts = {false, true};
    if (T.storage == LDPC_STORE_LDS) c2v_opts = {false};
    else if (T.storage != LDPC_STORE_AUTO) c2v_opts = {true};
    bool found = false;
    int best_fpc = 0;
    for (int tp : tps) {
      const int topo_b = align16((int)topo_bytes(c, tp));
      for (bool g : c2v_opts) {
        const int frame = align16(c->N * 4) + align16(syn) + (g ? 0 : align16(c->E * msg));
        if (topo_b + frame > pl.lds_limit) continue;
        int wpb = T.block ? T.block / WAVE : std::min(16, (160 * 1024 - topo_b) / frame);
        wpb = std::max(1, std::min(wpb, 16));
        while (wpb > 1 && topo_b + wpb * frame > pl.lds_limit) --wpb;
        const int lds = topo_b + wpb * frame;
        const int wgs = std::max(1, std::min((160 * 1024) / lds, 32 / wpb));
        int fpc = wgs * wpb;
        if (T.frames_per_cu) fpc = std::min(fpc, std::max(wpb, T.frames_per_cu / wpb * wpb));
        if (!found || fpc > best_fpc) {
          found = true;
          best_fpc = fpc;
          pl.topo = tp;
          pl.store = g ? STORE_ALL_GLOBAL : STORE_LDS;
          P.off_topo = 0;
          P.frame_base = topo_b;
          P.frame_stride = frame;
          P.wpb = wpb;
          P.off_L = 0;
          P.off_syn = align16(c->N * 4);
          P.off_c2v = P.off_syn + align16(syn);
          P.lds_bytes = lds;
        }
      }
    }
    if (!found) return LDPC_ECAPACITY;
    pl.block = WAVE * P.wpb;
    pl.persistent = true;
    const long long wg_needed = (B + P.wpb - 1) / P.wpb;
    pl.grid = (int)std::min<long long>(wg_needed, (long long)ncu * std::max(1, best_fpc / P.wpb));
    pl.scratch_bytes = kQueueBytes;
    if (pl.store != STORE_LDS) pl.scratch_bytes += (size_t)pl.grid * P.wpb * c->E * msg;
    return LDPC_OK;
  }

  if (c->max_dv > WAVE - 1) return LDPC_EUNSUPPORTED;
  if (c->nbr_max_cnt > NBR_PMAX * WAVE) return LDPC_EUNSUPPORTED;
  const std::vector<int> topos = topo_choices(c, T.topology);
  if (topos.empty()) return LDPC_EUNSUPPORTED;
  // STORE_FRAME_ALL is the capacity fallback only: on the BG1-shaped Z=52 code its 24 resident
  // frames per CU decoded 2% fewer frames/s than 12 with the check keys in LDS (the update loop
  // is bound by the memory system there, not by latency)
  std::vector<int> stores = {STORE_LDS,          STORE_PRE_GLOBAL, STORE_ALL_GLOBAL, STORE_ALL_GLOBAL_LT,
                             STORE_FRAME_GLOBAL, STORE_FRAME_REC};
  if (T.storage == LDPC_STORE_LDS) stores = {STORE_LDS};
  if (T.storage == LDPC_STORE_GLOBAL) stores = {STORE_PRE_GLOBAL};
  if (T.storage == LDPC_STORE_GLOBAL_ALL) stores = {STORE_ALL_GLOBAL};
  if (T.storage == LDPC_STORE_GLOBAL_LT) stores = {STORE_ALL_GLOBAL_LT};
  if (T.storage == LDPC_STORE_GLOBAL_FRAME) stores = {STORE_FRAME_GLOBAL};
  if (T.storage == LDPC_STORE_GLOBAL_REC) stores = {STORE_FRAME_REC};
  if (T.storage == LDPC_STORE_GLOBAL_STATE) stores = {STORE_FRAME_ALL};
  // LMDRBP and sLMDRBP read the check keys for their first choice only and write no CI records:
  // keys in global memory cost them nothing afterwards, and the LDS they leave holds more resident
  // frames (BG1-shaped Z=52: 20 frames per CU against 14, +14% and +8% frames/s).  LMD-CIRBP,
  // which still writes a record per touched VN, lost 3% that way and keeps the keys in LDS.
  if (T.storage == LDPC_STORE_AUTO && (s->kind == LDPC_LMDRBP || s->kind == LDPC_SLMDRBP))
    stores.push_back(STORE_FRAME_ALL);
  const int lut_off = 257 * (fixed ? s->frac_bits : 0);

  if (me) {
    MeParams& Q = pl.me;
    Q.lmd = s->kind == LDPC_ME_LMD_CIRBP ? 1 : 0;
    Q.B = B;
    Q.max_updates = max_updates;
    Q.check_every = s->check_every;
    Q.llr = llr_in;
    Q.out = o;
    Q.qmax = qmax;
    Q.scale = scale;
    Q.lut_global = c->d_lut + lut_off;
    Q.n_p = s->n_p;
    Q.n_g = s->n_g;
    Q.fill = s->fill;
    Q.seed = s->seed;
    bool found = false;
    MeLayout Ly{};
    std::vector<bool> me_stores = {false, true};
    if (T.storage == LDPC_STORE_LDS) me_stores = {false};
    if (T.storage >= LDPC_STORE_GLOBAL) me_stores = {true};
    for (bool g : me_stores) {
      for (int tp : topos) {
        MeLayout cand = me_layout(c, fixed, g, tp, s->n_p, s->n_g, s->fill);
        if (cand.total <= pl.lds_limit) {
          Ly = cand;
          pl.store = g ? STORE_ALL_GLOBAL : STORE_LDS;
          pl.topo = tp;
          found = true;
          break;
        }
      }
      if (found) break;
    }
    if (!found) return LDPC_ECAPACITY;
    Q.off_c2v = Ly.off_c2v; Q.off_pre = Ly.off_pre; Q.off_L = Ly.off_L; Q.off_Lt = Ly.off_Lt; Q.off_D = Ly.off_D;
    Q.off_hist = Ly.off_hist; Q.off_synw = Ly.off_synw; Q.off_rowmark = Ly.off_rowmark; Q.off_vnmark = Ly.off_vnmark;
    Q.off_rows = Ly.off_rows; Q.off_sel = Ly.off_sel; Q.off_cand = Ly.off_cand; Q.off_misc = Ly.off_misc;
    Q.off_lut = Ly.off_lut; Q.off_topo = Ly.off_topo; Q.off_rows2 = Ly.off_rows2; Q.off_vnmulti = Ly.off_vnmulti;
    Q.off_mpref = Ly.off_mpref; Q.off_macc = Ly.off_macc;
    Q.lds_bytes = Ly.total;
    Q.rows_cap = Ly.rows_cap;
    Q.cand_cap = Ly.cand_cap;
    Q.prof = nullptr;
#ifdef LDPC_PROFILE
    if (const char* pp = std::getenv("LDPCCI_PROF")) Q.prof = (long long*)std::strtoull(pp, nullptr, 10);
#endif
    pl.which = 2;
    pl.block = T.block ? T.block : (c->N <= 256 ? 64 : (c->N <= 2048 ? 256 : 1024));
    const int lds_per_cu = 160 * 1024;
    if (pl.store != STORE_LDS || T.frames_per_cu) {
      const int fit = std::max(1, lds_per_cu / std::max(Q.lds_bytes, 1));
      const int per_cu = T.frames_per_cu ? std::min(T.frames_per_cu, fit) : fit;
      pl.grid = (int)std::min<long long>(B, (long long)ncu * per_cu);
    } else if (!fixed) {
      // one workgroup per frame, up to four rounds of the workgroups a CU holds (each holds a
      // global slot for its step changes)
      const int fit = std::max(1, lds_per_cu / std::max(Q.lds_bytes, 1));
      pl.grid = (int)std::min<long long>(B, 4LL * ncu * fit);
    } else {
      pl.grid = B;
    }
    // per workgroup: the (c2v, pre) pairs when they are not in LDS; in FP32 the step's changes of
    // the precomputed messages, one float per edge (summed per VN in a fixed order)
    const size_t per_wg = (pl.store != STORE_LDS ? (size_t)2 * c->E * (fixed ? 1 : 4) : 0) + (fixed ? 0 : (size_t)4 * c->E);
    pl.scratch_bytes = (size_t)std::max(pl.grid, 1) * per_wg;
    return LDPC_OK;
  }

  DynParams& P = pl.dyn;
  P.kind = s->kind;
  P.B = B;
  P.max_updates = max_updates;
  P.check_every = s->check_every;
  P.llr = llr_in;
  P.replay = replay;
  P.replay_len = replay_len;
  P.out = o;
  P.qmax = qmax;
  P.scale = scale;
  P.lut_global = c->d_lut + lut_off;
  P.n_p = s->n_p;
  P.n_g = s->n_g;
  P.fill = s->fill;
  P.seed = s->seed;
  if (fixed) {
    double g = round_half_away((double)s->gamma * 65534.0);
    P.gamma_bits = (uint32_t)std::min(g, 4294967295.0);
  } else {
    float g = s->gamma;
    std::memcpy(&P.gamma_bits, &g, 4);
  }
  // storage plan.  Every (message storage, topology source) pair that fits is scored by the frames
  // per CU it lets the batch keep resident (at most 32, the wave slots of a CU).  More resident
  // frames win: one update is a chain of dependent steps, so throughput comes from overlapping
  // frames, and moving state to global memory adds little latency (both values of an edge come in
  // the load round trips the update makes anyway).  Ties: for a batch that fits in one round on
  // the chip, the most state in LDS (lowest latency); otherwise all messages in global memory.
  // Topology ties: quasi-cyclic tables, then LDS copies, then global arrays.  One frame per
  // workgroup unless the tuning asks for more (frames of a workgroup share its LDS topology copy;
  // whether that pays depends on the code, so it is left to the autotuner).
  DynLayout Ly{};
  bool found = false;
  int best_eff = 0, best_pref = -1;
  const long long need = std::max<long long>(1, (B + ncu - 1) / ncu);
  const int cap_fpc = T.frames_per_cu ? T.frames_per_cu : 32;
  // workgroups of w frames a CU holds: by LDS, and by wavefront slots at the variant's register
  // count (4 SIMDs per CU)
  auto wgs_per_cu = [&](const DynLayout& ly, int st, int tp, int w) {
    const int by_lds = std::max(1, (160 * 1024) / std::max(ly.total, 1));
    const int wps = dynamic_waves_per_simd(fixed, st, tp, tp != TOPO_GLOBAL && w > 1, is_lmd(s->kind));
    const int by_waves = std::max(1, (4 * wps) / w);
    return std::min(by_lds, by_waves);
  };
  for (int st : stores) {
    for (int tp : topos) {
      const int w = T.block && tp != TOPO_GLOBAL ? T.block / WAVE : 1;  // frames share LDS topology only
      DynLayout cand = dyn_layout(c, fixed, st, tp, w);
      if (cand.total > pl.lds_limit) continue;
      const int fit = std::min(32, w * wgs_per_cu(cand, st, tp, w));
      const int eff = (int)std::min<long long>(std::min(fit, cap_fpc), need);
      // Store preference: one round on the chip: LDS > PRE_GLOBAL > ALL_GLOBAL > ALL_GLOBAL_LT >
      // FRAME_REC > FRAME_ALL > FRAME_GLOBAL; larger batches: ALL_GLOBAL > ALL_GLOBAL_LT >
      // FRAME_REC > FRAME_ALL > FRAME_GLOBAL > PRE_GLOBAL > LDS (the record layout moves one
      // cache line per touched VN where the split arrays move three; keys in LDS beat keys in
      // global memory at equal residency)
      static const int rank_small[kStores] = {6, 5, 4, 3, 0, 2, 1}, rank_large[kStores] = {0, 1, 6, 5, 2, 4, 3};
      const int st_pref = need <= 1 ? rank_small[st] : rank_large[st];
      const int tp_pref = tp == TOPO_QC ? 2 : (tp == TOPO_LDS ? 1 : 0);
      const int pref = st_pref * 4 + tp_pref;
      if (!found || eff > best_eff || (eff == best_eff && pref > best_pref)) {
        Ly = cand;
        pl.store = st;
        pl.topo = tp;
        best_eff = eff;
        best_pref = pref;
        found = true;
      }
    }
  }
  if (!found && T.storage == LDPC_STORE_AUTO) {  // nothing else fits: check keys to global memory too
    for (int tp : topos) {
      const int w = T.block && tp != TOPO_GLOBAL ? T.block / WAVE : 1;
      DynLayout cand = dyn_layout(c, fixed, STORE_FRAME_ALL, tp, w);
      if (cand.total > pl.lds_limit) continue;
      const int eff = (int)std::min<long long>(
          std::min(std::min(32, w * wgs_per_cu(cand, STORE_FRAME_ALL, tp, w)), cap_fpc), need);
      if (!found || eff > best_eff) {
        Ly = cand;
        pl.store = STORE_FRAME_ALL;
        pl.topo = tp;
        best_eff = eff;
        found = true;
      }
    }
  }
  if (!found) return LDPC_ECAPACITY;
  // A quasi-cyclic code whose frames left the (small) QC tables for global topology: let several
  // frames share one LDS copy of the tables if that keeps at least 90% of the residency (measured
  // on the BG1-shaped codes: 12 frames per CU with shared tables beat 13 with global topology by
  // 7% at Z=52; 4 against 5 lost 9% at Z=128)
  if (!T.block && !T.topology && pl.topo == TOPO_GLOBAL && !c->h_qc.empty() && best_eff > 1) {
    int best_w = 0, best_fit = 0;
    DynLayout best_ly{};
    for (int ww = 2; ww <= 16; ++ww) {
      DynLayout cand = dyn_layout(c, fixed, pl.store, TOPO_QC, ww);
      if (cand.total > pl.lds_limit) break;
      const int fit = std::min(32, ww * wgs_per_cu(cand, pl.store, TOPO_QC, ww));
      if (fit > best_fit) {
        best_fit = fit;
        best_w = ww;
        best_ly = cand;
      }
    }
    if (best_w && 10LL * std::min<long long>(std::min(best_fit, cap_fpc), need) >= 9LL * best_eff) {
      Ly = best_ly;
      pl.topo = TOPO_QC;
    }
  }
  P.off_c2v = Ly.off_c2v; P.off_pre = Ly.off_pre; P.off_L = Ly.off_L; P.off_Lt = Ly.off_Lt;
  P.off_D = Ly.off_D; P.off_ckey = Ly.off_ckey; P.off_dblk = Ly.off_dblk; P.off_cblk = Ly.off_cblk;
  P.off_dmask = Ly.off_dmask; P.off_cmask = Ly.off_cmask; P.off_syn = Ly.off_syn; P.off_v = Ly.off_v;
  P.off_grp = Ly.off_grp; P.off_lut = Ly.off_lut; P.off_topo = Ly.off_topo;
  P.lds_bytes = Ly.total;
  P.frame_base = Ly.frame_base;
  P.frame_stride = Ly.frame_stride;
  P.wpb = Ly.wpb;
  P.nbd = Ly.nbd; P.nbc = Ly.nbc; P.nbd_words = Ly.nbd_words; P.nbc_words = Ly.nbc_words;
  P.prof = nullptr;
#ifdef LDPC_PROFILE
  if (const char* pp = std::getenv("LDPCCI_PROF")) P.prof = (long long*)std::strtoull(pp, nullptr, 10);
#endif
  P.selfcheck = nullptr;
#ifdef LDPC_SELFCHECK
  if (const char* sp = std::getenv("LDPCCI_SELFCHECK")) P.selfcheck = (unsigned long long*)std::strtoull(sp, nullptr, 10);
#endif
  pl.which = 1;
  pl.block = WAVE * P.wpb;
  // persistent grid (workers pull frames from a queue) unless one workgroup per frame fills the
  // chip in a single round and the messages stay in LDS
  pl.persistent = pl.store != STORE_LDS || T.frames_per_cu || need > 1;
  const long long wg_needed = (B + P.wpb - 1) / P.wpb;
  if (pl.persistent) {
    const int wgs = wgs_per_cu(Ly, pl.store, pl.topo, P.wpb);
    const int wg_per_cu = std::max(1, std::min(wgs, std::min(32, cap_fpc) / P.wpb));
    pl.grid = (int)std::min<long long>(wg_needed, (long long)ncu * wg_per_cu);
  } else {
    pl.grid = (int)wg_needed;
  }
  const size_t msg = fixed ? 1 : 4;
  const size_t slots = (size_t)std::max(pl.grid, 1) * P.wpb;
  if (pl.persistent) pl.scratch_bytes = kQueueBytes;  // work-queue counter, then message slots
  if (pl.store == STORE_PRE_GLOBAL) pl.scratch_bytes += slots * c->E * msg;
  if (pl.store >= STORE_ALL_GLOBAL) {
    all_global_slot(c->E, c->N, c->M, (c->nbr_max_cnt + WAVE - 1) / WAVE, fixed, pl.store, P);
    pl.scratch_bytes += slots * (size_t)P.slot_bytes;
  }
  return LDPC_OK;
}

// Raise the kernels' dynamic-LDS limit for a plan (not a stream operation: done before capture).
hipError_t plan_lds_limits(const DecodePlan& pl) {
  if (pl.which == 0) return raise_lds_limit(FAM_BASELINE, pl.lds_limit, set_baseline_lds_limit);
  if (pl.which == 2) return raise_lds_limit(FAM_ME, pl.lds_limit, set_me_lds_limit);
  return raise_lds_limit(FAM_DYNAMIC, pl.lds_limit, set_dynamic_lds_limit);
}

// Enqueue a planned decode; scratch must hold pl.scratch_bytes (may be null when that is 0).
// With set_attr false the caller has applied plan_lds_limits already (stream capture).
hipError_t enqueue_decode(const ldpc_code* c, DecodePlan& pl, void* scratch, hipStream_t st, bool set_attr = true) {
  if (pl.grid <= 0) return hipSuccess;
  if (injected_fault() == FAULT_LAUNCH) return hipErrorLaunchFailure;
  if (set_attr) {
    hipError_t he = plan_lds_limits(pl);
    if (he != hipSuccess) return he;
  }
  if (pl.which == 0) {
    if (pl.persistent) {
      pl.base.queue = reinterpret_cast<int*>(scratch);
      pl.base.c2v_global = pl.store != STORE_LDS ? (char*)scratch + kQueueBytes : nullptr;
      hipError_t he = launch_fill_u64(reinterpret_cast<int64_t*>(scratch), 1, 0, st);  // queue = 0
      if (he != hipSuccess) return he;
    }
    return launch_baseline(c->dev, pl.base, pl.fixed, pl.topo, pl.grid, pl.block, st);
  }
  if (pl.which == 2) {
    const bool mg = pl.store != STORE_LDS;
    pl.me.msg_global = mg ? scratch : nullptr;
    pl.me.dbuf = pl.fixed ? nullptr
                          : reinterpret_cast<float*>((char*)scratch + (mg ? (size_t)pl.grid * 2 * c->E * 4 : 0));
    return launch_me(c->dev, pl.me, pl.fixed, mg, pl.topo, pl.grid, pl.block, st);
  }
  pl.dyn.queue = pl.persistent ? reinterpret_cast<int*>(scratch) : nullptr;
  pl.dyn.pre_global = pl.store != STORE_LDS ? (char*)scratch + kQueueBytes : nullptr;
  if (pl.persistent) {
    hipError_t he = launch_fill_u64(reinterpret_cast<int64_t*>(scratch), 1, 0, st);  // queue = 0
    if (he != hipSuccess) return he;
  }
  return launch_dynamic(c->dev, pl.dyn, pl.fixed, pl.store, pl.topo, pl.grid, st);
}

// ------------------------------------------------------------------------------------------
// tuning table: process-wide, keyed by (code signature, schedule kind, arithmetic)
// ------------------------------------------------------------------------------------------
struct TuneKey {
  uint64_t sig;
  int kind, arith;
  bool operator<(const TuneKey& o) const {
    if (sig != o.sig) return sig < o.sig;
    if (kind != o.kind) return kind < o.kind;
    return arith < o.arith;
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, ldpc_tuning> g_tune;

// process-wide tuning of ldpc_decode_batch (storage and frames per CU; block must be 0)
std::mutex g_btune_mu;
bool g_btune_set = false;
ldpc_tuning g_btune{};

int check_batch_tuning(const ldpc_tuning* t) {
  if (!t) return LDPC_OK;
  if (int rc = check_tuning(t)) return rc;
  if (t->block != 0 || t->topology != LDPC_TOPO_AUTO) return LDPC_EINVAL;
  if (t->storage == LDPC_STORE_GLOBAL_STATE) return LDPC_EUNSUPPORTED;  // no batched variant
  return LDPC_OK;
}


bool lookup_tuning(const ldpc_code* c, int kind, int arith, ldpc_tuning& t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(TuneKey{c->sig, kind, arith});
  if (it == g_tune.end()) return false;
  t = it->second;
  return true;
}

}  // namespace

extern "C" {

int ldpc_decode(const ldpc_code* c, const ldpc_schedule* s, const float* llr_in, int32_t B, int64_t max_updates,
                const int32_t* replay, int64_t replay_len, const ldpc_outputs* out, void* stream) {
  if (!c || !s || !out || B < 0 || max_updates < 0) return LDPC_EINVAL;
  if (B == 0) return LDPC_OK;
  ldpc_tuning t{};
  const bool tuned = lookup_tuning(c, s->kind, s->arith, t);
  DecodePlan pl;
  int rc = plan_decode(c, s, llr_in, B, max_updates, replay, replay_len, out, tuned ? &t : nullptr, pl);
  if (rc != LDPC_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  void* scratch = nullptr;
  if (pl.scratch_bytes) {
    hipError_t he = scratch_alloc(&scratch, pl.scratch_bytes, st);
    if (he != hipSuccess) return he == hipErrorOutOfMemory ? LDPC_ENOMEM : hip_fail(he);
  }
  hipError_t he = enqueue_decode(c, pl, scratch, st);
  if (scratch) (void)hipFreeAsync(scratch, st);
  return he == hipSuccess ? LDPC_OK : hip_fail(he);
}

}  // extern "C"

namespace {

// Shrink a plan's persistent grid until its scratch fits cap bytes.  Workers take frames from a
// queue (single-edge) or in strides of the grid (ME), so any grid of at least one workgroup decodes
// every frame, with the same per-frame outputs; fewer workers only lower throughput.
int fit_plan_to_scratch(const ldpc_code* c, DecodePlan& pl, size_t cap) {
  if (pl.scratch_bytes <= cap) return LDPC_OK;
  size_t head = 0, per_wg = 0;
  if (pl.which == 0 && pl.persistent) {
    head = kQueueBytes;
    if (pl.store != STORE_LDS) per_wg = (size_t)pl.base.wpb * c->E * (pl.fixed ? 1 : 4);
  } else if (pl.which == 1) {
    head = pl.persistent ? kQueueBytes : 0;
    const size_t msg = pl.fixed ? 1 : 4;
    if (pl.store == STORE_PRE_GLOBAL) per_wg = (size_t)pl.dyn.wpb * c->E * msg;
    else if (pl.store >= STORE_ALL_GLOBAL) per_wg = (size_t)pl.dyn.wpb * (size_t)pl.dyn.slot_bytes;
  } else if (pl.which == 2) {
    per_wg = (pl.store != STORE_LDS ? (size_t)2 * c->E * (pl.fixed ? 1 : 4) : 0) + (pl.fixed ? 0 : (size_t)4 * c->E);
  }
  if (per_wg == 0 || cap < head + per_wg) return LDPC_ECAPACITY;
  const size_t grid = std::min<size_t>((size_t)pl.grid, (cap - head) / per_wg);
  pl.grid = (int)grid;
  pl.scratch_bytes = head + grid * per_wg;
  return LDPC_OK;
}

}  // namespace

namespace ldpc {

int record_hip_failure(hipError_t e) { return hip_fail(e); }

const int* abort_flag_address() {
  std::lock_guard<std::mutex> lk(g_abort_mu);
  return g_abort_dev;
}

int decode_in_scratch(const ldpc_code* c, const ldpc_schedule* s, const float* llr_in, int32_t B,
                      int64_t max_updates, const int32_t* replay, int64_t replay_len, const ldpc_outputs* out,
                      void* scratch, size_t cap, hipStream_t st) {
  if (!c || !s || !out || B < 0 || max_updates < 0) return LDPC_EINVAL;
  if (B == 0) return LDPC_OK;
  ldpc_tuning t{};
  const bool tuned = lookup_tuning(c, s->kind, s->arith, t);
  DecodePlan pl;
  int rc = plan_decode(c, s, llr_in, B, max_updates, replay, replay_len, out, tuned ? &t : nullptr, pl);
  if (rc != LDPC_OK) return rc;
  if ((rc = fit_plan_to_scratch(c, pl, cap)) != LDPC_OK) return rc;
  const hipError_t he = enqueue_decode(c, pl, pl.scratch_bytes ? scratch : nullptr, st);
  return he == hipSuccess ? LDPC_OK : hip_fail(he);
}

}  // namespace ldpc

extern "C" {

int ldpc_describe_plan(const ldpc_code* c, const ldpc_schedule* s, int32_t B, ldpc_plan_info* info) {
  if (!c || !s || !info || B < 1) return LDPC_EINVAL;
  ldpc_tuning t{};
  const bool tuned = lookup_tuning(c, s->kind, s->arith, t);
  DecodePlan pl;
  int rc = plan_decode(c, s, nullptr, B, 0, nullptr, 0, nullptr, tuned ? &t : nullptr, pl, true);
  if (rc != LDPC_OK) return rc;
  ldpc_plan_info r{};
  r.kernel = pl.which;
  r.storage = pl.store + 1;  // Store -> LDPC_STORE_* (shifted by AUTO)
  r.topology = pl.topo + 1;
  r.block = pl.block;
  r.grid = pl.grid;
  r.frames_per_workgroup = pl.which == 1 ? pl.dyn.wpb : (pl.which == 0 ? pl.base.wpb : 1);
  const int lds = pl.which == 0 ? pl.base.lds_bytes : (pl.which == 1 ? pl.dyn.lds_bytes : pl.me.lds_bytes);
  const int by_lds = std::max(1, (160 * 1024) / std::max(lds, 1));
  const int wps = pl.which == 1 ? dynamic_waves_per_simd(pl.fixed, pl.store, pl.topo, pl.topo != TOPO_GLOBAL && pl.dyn.wpb > 1,
                                                       is_lmd(pl.dyn.kind))
                                : 8;
  const int by_waves = std::max(1, 4 * wps / std::max(1, pl.block / WAVE));
  r.workgroups_per_cu = std::min(by_lds, by_waves);
  r.persistent = pl.which <= 1 ? (pl.persistent ? 1 : 0) : (pl.grid < B ? 1 : 0);
  r.lds_bytes = lds;
  r.scratch_bytes = (int64_t)pl.scratch_bytes;
  *info = r;
  return LDPC_OK;
}

int ldpc_set_tuning(const ldpc_code* c, int32_t kind, int32_t arith, const ldpc_tuning* t) {
  if (!c || kind < LDPC_FLOODING || kind > LDPC_ME_LMD_CIRBP || (arith != LDPC_SPA_F32 && arith != LDPC_MS_FIX))
    return LDPC_EINVAL;
  if (int rc = check_tuning(t)) return rc;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (t) g_tune[TuneKey{c->sig, kind, arith}] = *t;
  else g_tune.erase(TuneKey{c->sig, kind, arith});
  return LDPC_OK;
}

int ldpc_get_tuning(const ldpc_code* c, int32_t kind, int32_t arith, ldpc_tuning* out) {
  if (!c || !out) return LDPC_EINVAL;
  ldpc_tuning t{};
  const bool found = lookup_tuning(c, kind, arith, t);
  *out = t;
  return found ? 1 : 0;
}

int ldpc_autotune(const ldpc_code* c, const ldpc_schedule* s, const float* llr_in, int32_t B, int64_t max_updates,
                  int32_t reps, ldpc_tuning* best, float* best_ms, void* stream) {
  if (!c || !s || !llr_in || B < 1 || max_updates < 0 || reps < 1 || reps > 100) return LDPC_EINVAL;
  if (s->kind == LDPC_REPLAY) return LDPC_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  // candidate knobs of the kernel family this schedule runs on
  std::vector<ldpc_tuning> cands;
  if (s->kind == LDPC_FLOODING) {
    for (int b : {64, 128, 256, 512, 1024}) cands.push_back(ldpc_tuning{b, 0, 0, 0});
  } else if (s->kind == LDPC_LAYERED) {  // frames per workgroup x c2v in LDS or in a global slot
    for (int b : {0, 64, 256, 512, 1024})
      for (int store : {LDPC_STORE_AUTO, LDPC_STORE_LDS, LDPC_STORE_GLOBAL_ALL}) cands.push_back(ldpc_tuning{b, 0, store, 0});
  } else {
    std::vector<int> tps = {LDPC_TOPO_GLOBAL, LDPC_TOPO_LDS};
    if (!c->h_qc.empty()) tps.push_back(LDPC_TOPO_QC);
    const bool me = s->kind == LDPC_ME_CIRBP || s->kind == LDPC_ME_LMD_CIRBP;
    const std::vector<int> blocks = me ? std::vector<int>{64, 256, 1024} : std::vector<int>{0};
    for (int b : blocks)
      for (int store : {LDPC_STORE_LDS, LDPC_STORE_GLOBAL, LDPC_STORE_GLOBAL_ALL, LDPC_STORE_GLOBAL_LT,
                        LDPC_STORE_GLOBAL_FRAME, LDPC_STORE_GLOBAL_REC, LDPC_STORE_GLOBAL_STATE})
        for (int tp : tps)
          for (int fpc : {0, 1, 2, 4, 8, 16})
            for (int wb : me ? std::vector<int>{0} : std::vector<int>{0, 256, 512})
              cands.push_back(ldpc_tuning{me ? b : wb, fpc, store, tp});
  }
  // outputs for the trial decodes (discarded)
  uint8_t* bits = nullptr;
  int64_t* upd = nullptr;
  hipError_t he = hipMalloc((void**)&bits, (size_t)B * c->N);
  if (he == hipSuccess) he = hipMalloc((void**)&upd, (size_t)B * sizeof(int64_t));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (he == hipSuccess) he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  int rc = LDPC_OK;
  float best_t = -1.0f;
  ldpc_tuning best_c{};
  for (size_t i = 0; i < cands.size() && he == hipSuccess && rc == LDPC_OK; ++i) {
    ldpc_outputs out{};
    out.bits = bits;
    out.updates_used = upd;
    DecodePlan pl;
    if (plan_decode(c, s, llr_in, B, max_updates, nullptr, 0, &out, &cands[i], pl) != LDPC_OK) continue;
    // skip knobs that resolve to a plan already timed
    bool dup = false;
    for (size_t j = 0; j < i && !dup; ++j) {
      DecodePlan q;
      if (plan_decode(c, s, llr_in, B, max_updates, nullptr, 0, &out, &cands[j], q) != LDPC_OK) continue;
      dup = q.which == pl.which && q.grid == pl.grid && q.block == pl.block && q.topo == pl.topo &&
            q.store == pl.store && q.persistent == pl.persistent;
    }
    if (dup) continue;
    void* scratch = nullptr;
    if (pl.scratch_bytes && (he = hipMalloc(&scratch, pl.scratch_bytes)) != hipSuccess) {
      if (he != hipErrorOutOfMemory) break;
      (void)hipGetLastError();  // a plan whose scratch does not fit is skipped, not fatal
      he = hipSuccess;
      continue;
    }
    float tmin = -1.0f;
    he = enqueue_decode(c, pl, scratch, st);  // warm-up
    for (int r = 0; r < reps && he == hipSuccess; ++r) {
      he = hipEventRecord(e0, st);
      if (he == hipSuccess) he = enqueue_decode(c, pl, scratch, st);
      if (he == hipSuccess) he = hipEventRecord(e1, st);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he == hipSuccess && (tmin < 0.0f || ms < tmin)) tmin = ms;
    }
    if (scratch) (void)hipFree(scratch);
    if (he == hipSuccess && tmin >= 0.0f && (best_t < 0.0f || tmin < best_t)) {
      best_t = tmin;
      best_c = cands[i];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (bits) (void)hipFree(bits);
  if (upd) (void)hipFree(upd);
  if (he != hipSuccess) return hip_fail(he);
  if (best_t < 0.0f) return LDPC_ECAPACITY;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[TuneKey{c->sig, s->kind, s->arith}] = best_c;
  }
  if (best) *best = best_c;
  if (best_ms) *best_ms = best_t;
  return rc;
}

int ldpc_tuning_save(const char* path) {
  if (!path) return LDPC_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LDPC_EHIP;
  const std::string tag = device_tag(dev);
  FILE* f = std::fopen(path, "w");
  if (!f) return LDPC_EINVAL;
  ldpc_tuning bt{};
  bool bset = false;
  {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    bset = g_btune_set;
    bt = g_btune;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::fprintf(f, "{\"device\": \"%s\", \"entries\": [\n", tag.c_str());
  const size_t count = g_tune.size() + (bset ? 1 : 0);
  size_t i = 0;
  for (const auto& kv : g_tune) {
    const ldpc_tuning& t = kv.second;
    std::fprintf(f,
                 "{\"sig\": \"%016llx\", \"kind\": %d, \"arith\": %d, \"block\": %d, \"frames_per_cu\": %d, "
                 "\"storage\": %d, \"topology\": %d}%s\n",
                 (unsigned long long)kv.first.sig, kv.first.kind, kv.first.arith, t.block, t.frames_per_cu, t.storage,
                 t.topology, ++i < count ? "," : "");
  }
  if (bset)  // the batched launch's tuning (ldpc_set_batch_tuning)
    std::fprintf(f, "{\"batch\": 1, \"frames_per_cu\": %d, \"storage\": %d}\n", bt.frames_per_cu, bt.storage);
  std::fprintf(f, "]}\n");
  return std::fclose(f) == 0 ? LDPC_OK : LDPC_EINVAL;
}

int ldpc_tuning_load(const char* path) {
  if (!path) return LDPC_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LDPC_EHIP;
  const std::string tag = device_tag(dev);
  FILE* f = std::fopen(path, "r");
  if (!f) return LDPC_EINVAL;
  char line[512];
  int loaded = 0;
  bool same_device = false;
  std::vector<std::pair<TuneKey, ldpc_tuning>> rows;
  ldpc_tuning batch{};
  bool have_batch = false;
  while (std::fgets(line, sizeof line, f)) {
    char dtag[128];
    if (std::sscanf(line, " {\"device\": \"%127[^\"]\"", dtag) == 1) {
      same_device = tag == dtag;
      continue;
    }
    int bfpc = 0, bst = 0;
    if (std::sscanf(line, " {\"batch\": 1, \"frames_per_cu\": %d, \"storage\": %d}", &bfpc, &bst) == 2) {
      const ldpc_tuning bt{0, bfpc, bst, LDPC_TOPO_AUTO};
      if (check_batch_tuning(&bt) == LDPC_OK) {
        batch = bt;
        have_batch = true;
      }
      continue;
    }
    unsigned long long sig = 0;
    TuneKey k{};
    ldpc_tuning t{};
    if (std::sscanf(line,
                    " {\"sig\": \"%llx\", \"kind\": %d, \"arith\": %d, \"block\": %d, \"frames_per_cu\": %d, "
                    "\"storage\": %d, \"topology\": %d}",
                    &sig, &k.kind, &k.arith, &t.block, &t.frames_per_cu, &t.storage, &t.topology) == 7) {
      k.sig = sig;
      if (check_tuning(&t) != LDPC_OK || k.kind < LDPC_FLOODING || k.kind > LDPC_ME_LMD_CIRBP) continue;
      rows.push_back({k, t});
    }
  }
  std::fclose(f);
  if (!same_device) return 0;
  if (have_batch) {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    g_btune_set = true;
    g_btune = batch;
    ++loaded;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& r : rows) {
    g_tune[r.first] = r.second;
    ++loaded;
  }
  return loaded;
}

}  // extern "C"

namespace {

// ldpc_decode_batch with an explicit tuning (nullable: the default policy)
// A batched launch resolved: storage mode, topology source, LDS layout of the largest code,
// resident frames per CU, grid and scratch bytes.
struct BatchPlan {
  bool fixed = false;
  int store = -1, topo = TOPO_GLOBAL, per_cu = 0, grid = 0, lds_limit = 0;
  Dims mx{0, 0, 0, 0, 0};
  DynLayout Ly{};
  size_t pre_bytes = 0;
  DynParams slot{};  // slot offsets when the frame state is global
};

int plan_batch(const ldpc_code* const* codes, int32_t n_codes, const ldpc_schedule* s, int32_t F,
               const ldpc_tuning* T, BatchPlan& bp) {
  if (!codes || n_codes < 1 || n_codes > 64 || !s || F < 0) return LDPC_EINVAL;
  if (int rc = check_batch_tuning(T)) return rc;
  if (s->arith != LDPC_SPA_F32 && s->arith != LDPC_MS_FIX) return LDPC_EINVAL;
  bp = BatchPlan{};
  bp.fixed = s->arith == LDPC_MS_FIX;
  if (bp.fixed && (s->q_bits < 2 || s->q_bits > 8 || s->frac_bits < 0 || s->frac_bits > 6)) return LDPC_EINVAL;
  if (s->check_every < 0) return LDPC_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LDPC_EHIP;
  bool all_qc = true;
  Dims& mx = bp.mx;
  for (int i = 0; i < n_codes; ++i) {
    const ldpc_code* c = codes[i];
    if (!c || c->device != dev) return LDPC_EINVAL;
    if (c->max_dv > WAVE - 1 || c->nbr_max_cnt > NBR_PMAX * WAVE) return LDPC_EUNSUPPORTED;
    all_qc = all_qc && !c->h_qc.empty();
    mx.E = std::max(mx.E, c->E);
    mx.N = std::max(mx.N, c->N);
    mx.M = std::max(mx.M, c->M);
    mx.nbr_passes = std::max(mx.nbr_passes, (c->nbr_max_cnt + WAVE - 1) / WAVE);
  }
  bp.topo = all_qc ? TOPO_QC : TOPO_GLOBAL;
  for (int i = 0; i < n_codes; ++i) mx.topo_bytes = std::max(mx.topo_bytes, topo_bytes(codes[i], bp.topo));
  bp.lds_limit = std::min(device_lds_limit(dev), 160 * 1024);
  const int ncu = device_cu_count(dev);
  // message storage: the mode that keeps the most frames resident per CU (at most 32); ties go to
  // the later mode of the list (the batch is a large persistent launch: messages global, then VN
  // records over split arrays)
  int best_fit = 0;
  for (int st : {STORE_LDS, STORE_PRE_GLOBAL, STORE_FRAME_GLOBAL, STORE_FRAME_REC, STORE_ALL_GLOBAL_LT, STORE_ALL_GLOBAL}) {
    if (T && T->storage != LDPC_STORE_AUTO && st != T->storage - 1) continue;  // LDPC_STORE_* = Store + 1
    DynLayout cand = dyn_layout_dims(mx, bp.fixed, st, 1);
    if (cand.total > bp.lds_limit) continue;
    const int fit = std::min(32, (160 * 1024) / std::max(cand.total, 1));
    if (bp.store < 0 || fit >= best_fit) {
      bp.store = st;
      best_fit = fit;
      bp.Ly = cand;
    }
  }
  if (bp.store < 0) return LDPC_ECAPACITY;
  bp.per_cu = std::max(1, std::min(32, (160 * 1024) / std::max(bp.Ly.total, 1)));
  if (T && T->frames_per_cu) bp.per_cu = std::min(bp.per_cu, T->frames_per_cu);
  bp.grid = (int)std::min<long long>(std::max(F, 1), (long long)ncu * bp.per_cu);
  // scratch: the work-queue counter and the frame slots if needed
  if (bp.store == STORE_PRE_GLOBAL) bp.pre_bytes = (size_t)bp.grid * mx.E * (bp.fixed ? 1 : 4);
  if (bp.store >= STORE_ALL_GLOBAL) {
    all_global_slot(mx.E, mx.N, mx.M, mx.nbr_passes, bp.fixed, bp.store, bp.slot);
    bp.pre_bytes = (size_t)bp.grid * (size_t)bp.slot.slot_bytes;
  }
  return LDPC_OK;
}

// ldpc_decode_batch with an explicit tuning (nullable: the default policy)
int decode_batch_tuned(const ldpc_code* const* codes, int32_t n_codes, const ldpc_schedule* s,
                       const ldpc_frame_desc* frames, int32_t F, const float* llr_pool, int64_t llr_len,
                       uint8_t* bits_pool, float* llr_out_pool, int64_t out_len, int64_t* updates_used,
                       int64_t* steps_used, int64_t* fallbacks, void* stream, const ldpc_tuning* T) {
  static_assert(sizeof(ldpc_frame_desc) == sizeof(BatchFrame), "descriptor layout");
  if (!codes || n_codes < 1 || n_codes > 64 || !s || F < 0 || llr_len < 0 || out_len < 0) return LDPC_EINVAL;
  if (int rc = check_batch_tuning(T)) return rc;
  if (F == 0) return LDPC_OK;
  if (!frames || !llr_pool || !bits_pool || !updates_used) return LDPC_EINVAL;
  BatchPlan bp;
  if (int rc = plan_batch(codes, n_codes, s, F, T, bp)) return rc;
  const bool fixed = bp.fixed;
  const DynLayout& Ly = bp.Ly;
  hipStream_t st = (hipStream_t)stream;
  BatchParams B{};
  DynParams& P = B.P;
#ifdef LDPC_SELFCHECK
  if (const char* sp = std::getenv("LDPCCI_SELFCHECK")) P.selfcheck = (unsigned long long*)std::strtoull(sp, nullptr, 10);
#endif
  P.check_every = s->check_every;
  P.qmax = (1 << (std::max(s->q_bits, 2) - 1)) - 1;
  P.scale = std::ldexp(1.0f, fixed ? s->frac_bits : 0);
  P.lut_global = codes[0]->d_lut + 257 * (fixed ? s->frac_bits : 0);
  P.off_c2v = Ly.off_c2v; P.off_pre = Ly.off_pre; P.off_L = Ly.off_L; P.off_Lt = Ly.off_Lt;
  P.off_D = Ly.off_D; P.off_ckey = Ly.off_ckey; P.off_dblk = Ly.off_dblk; P.off_cblk = Ly.off_cblk;
  P.off_dmask = Ly.off_dmask; P.off_cmask = Ly.off_cmask; P.off_syn = Ly.off_syn; P.off_v = Ly.off_v;
  P.off_grp = Ly.off_grp; P.off_lut = Ly.off_lut; P.off_topo = Ly.off_topo;
  P.lds_bytes = Ly.total;
  P.frame_base = Ly.frame_base;
  P.frame_stride = Ly.frame_stride;
  P.wpb = 1;
  if (bp.store >= STORE_ALL_GLOBAL) {
    P.slot_bytes = bp.slot.slot_bytes;
    P.slot_lt_off = bp.slot.slot_lt_off;
    P.slot_l_off = bp.slot.slot_l_off;
    P.slot_d_off = bp.slot.slot_d_off;
    P.slot_ckey_off = bp.slot.slot_ckey_off;
    P.slot_tj_off = bp.slot.slot_tj_off;
  }
  B.n_codes = n_codes;
  B.frames = reinterpret_cast<const BatchFrame*>(frames);
  B.F = F;
  B.llr_pool = llr_pool;
  B.llr_len = llr_len;
  B.bits_pool = bits_pool;
  B.llr_out_pool = llr_out_pool;
  B.out_len = out_len;
  B.updates_used = updates_used;
  B.steps_used = steps_used;
  B.fallbacks = fallbacks;
  B.max_E = bp.mx.E;
  B.abort = ldpc::abort_flag_address();
  void* scratch = nullptr;
  hipError_t he = scratch_alloc(&scratch, 256 + bp.pre_bytes, st);
  if (he != hipSuccess) return he == hipErrorOutOfMemory ? LDPC_ENOMEM : hip_fail(he);
  for (int i = 0; i < n_codes; ++i) B.codes[i] = codes[i]->d_self;
  B.queue = reinterpret_cast<int*>(scratch);
  P.pre_global = bp.store != STORE_LDS ? (char*)scratch + 256 : nullptr;
  he = raise_lds_limit(FAM_BATCH, bp.lds_limit, set_batch_lds_limit);
  if (he == hipSuccess && injected_fault() == FAULT_LAUNCH) he = hipErrorLaunchFailure;
  if (he == hipSuccess) he = launch_batch(B, fixed, bp.store, bp.topo, bp.grid, st);
  (void)hipFreeAsync(scratch, st);
  return he == hipSuccess ? LDPC_OK : hip_fail(he);
}

}  // namespace

extern "C" {

int ldpc_decode_batch(const ldpc_code* const* codes, int32_t n_codes, const ldpc_schedule* s,
                      const ldpc_frame_desc* frames, int32_t F, const float* llr_pool, int64_t llr_len,
                      uint8_t* bits_pool, float* llr_out_pool, int64_t out_len, int64_t* updates_used,
                      int64_t* steps_used, int64_t* fallbacks, void* stream) {
  ldpc_tuning t{};
  bool tuned = false;
  {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    tuned = g_btune_set;
    t = g_btune;
  }
  return decode_batch_tuned(codes, n_codes, s, frames, F, llr_pool, llr_len, bits_pool, llr_out_pool, out_len,
                            updates_used, steps_used, fallbacks, stream, tuned ? &t : nullptr);
}

int ldpc_describe_batch_plan(const ldpc_code* const* codes, int32_t n_codes, const ldpc_schedule* s, int32_t F,
                             ldpc_plan_info* info) {
  if (!info || F < 1) return LDPC_EINVAL;
  ldpc_tuning t{};
  bool tuned = false;
  {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    tuned = g_btune_set;
    t = g_btune;
  }
  BatchPlan bp;
  if (int rc = plan_batch(codes, n_codes, s, F, tuned ? &t : nullptr, bp)) return rc;
  ldpc_plan_info r{};
  r.kernel = 3;
  r.storage = bp.store + 1;
  r.topology = bp.topo + 1;
  r.block = WAVE;
  r.grid = bp.grid;
  r.frames_per_workgroup = 1;
  r.workgroups_per_cu = bp.per_cu;
  r.persistent = 1;
  r.lds_bytes = bp.Ly.total;
  r.scratch_bytes = (int64_t)(256 + bp.pre_bytes);
  *info = r;
  return LDPC_OK;
}

int ldpc_set_batch_tuning(const ldpc_tuning* t) {
  if (int rc = check_batch_tuning(t)) return rc;
  std::lock_guard<std::mutex> lk(g_btune_mu);
  g_btune_set = t != nullptr;
  g_btune = t ? *t : ldpc_tuning{};
  return LDPC_OK;
}

int ldpc_get_batch_tuning(ldpc_tuning* out) {
  if (!out) return LDPC_EINVAL;
  std::lock_guard<std::mutex> lk(g_btune_mu);
  *out = g_btune;
  return g_btune_set ? 1 : 0;
}

int ldpc_autotune_batch(const ldpc_code* const* codes, int32_t n_codes, const ldpc_schedule* s,
                        const ldpc_frame_desc* frames, int32_t F, const float* llr_pool, int64_t llr_len,
                        int64_t out_len, int32_t reps, ldpc_tuning* best, float* best_ms, void* stream) {
  if (F < 1 || out_len < 0 || reps < 1 || reps > 100) return LDPC_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  // trial outputs (discarded)
  uint8_t* bits = nullptr;
  int64_t* upd = nullptr;
  hipError_t he = hipMalloc((void**)&bits, (size_t)std::max<int64_t>(out_len, 1));
  if (he == hipSuccess) he = hipMalloc((void**)&upd, (size_t)F * sizeof(int64_t));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (he == hipSuccess) he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  float best_t = -1.0f;
  ldpc_tuning best_c{};
  int rc = LDPC_OK;
  for (int store : {LDPC_STORE_AUTO, LDPC_STORE_LDS, LDPC_STORE_GLOBAL, LDPC_STORE_GLOBAL_ALL, LDPC_STORE_GLOBAL_LT,
                    LDPC_STORE_GLOBAL_FRAME, LDPC_STORE_GLOBAL_REC}) {
    for (int fpc : {0, 4, 8, 12, 16, 24}) {
      if (he != hipSuccess) break;
      const ldpc_tuning cand{0, fpc, store, LDPC_TOPO_AUTO};
      auto run = [&]() {
        return decode_batch_tuned(codes, n_codes, s, frames, F, llr_pool, llr_len, bits, nullptr, out_len, upd,
                                  nullptr, nullptr, stream, &cand);
      };
      const int r0 = run();  // warm-up; a candidate whose state does not fit is skipped
      if (r0 == LDPC_ECAPACITY || r0 == LDPC_ENOMEM) continue;
      if (r0 != LDPC_OK) {
        rc = r0;
        break;
      }
      float tmin = -1.0f;
      for (int r = 0; r < reps && he == hipSuccess && rc == LDPC_OK; ++r) {
        he = hipEventRecord(e0, st);
        if (he == hipSuccess) rc = run();
        if (he == hipSuccess && rc == LDPC_OK) he = hipEventRecord(e1, st);
        if (he == hipSuccess && rc == LDPC_OK) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess && rc == LDPC_OK) he = hipEventElapsedTime(&ms, e0, e1);
        if (he == hipSuccess && rc == LDPC_OK && (tmin < 0.0f || ms < tmin)) tmin = ms;
      }
      if (rc != LDPC_OK) break;
      if (he == hipSuccess && tmin >= 0.0f && (best_t < 0.0f || tmin < best_t)) {
        best_t = tmin;
        best_c = cand;
      }
    }
    if (rc != LDPC_OK || he != hipSuccess) break;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (bits) (void)hipFree(bits);
  if (upd) (void)hipFree(upd);
  if (he != hipSuccess) return hip_fail(he);
  if (rc != LDPC_OK) return rc;
  if (best_t < 0.0f) return LDPC_ECAPACITY;
  {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    g_btune_set = true;
    g_btune = best_c;
  }
  if (best) *best = best_c;
  if (best_ms) *best_ms = best_t;
  return LDPC_OK;
}

// ------------------------------------------------------------------------------------------
// differentiable unrolled decoder
// ------------------------------------------------------------------------------------------
static int unroll_check(const ldpc_code* c, int32_t B, int32_t T, int32_t K, int* dev) {
  if (!c || B < 0 || T < 0 || K < 1 || K > LDPC_UNROLL_MAX_CKPT_EVERY) return LDPC_EINVAL;
  if (hipGetDevice(dev) != hipSuccess) return LDPC_EHIP;
  if (c->device != *dev) return LDPC_EINVAL;
  if (c->min_dc < 2 || c->max_dc > 32) return LDPC_EUNSUPPORTED;
  return LDPC_OK;
}

int64_t ldpc_unrolled_ckpt_floats(const ldpc_code* c, int32_t T, int32_t ckpt_every) {
  if (!c || T < 0 || ckpt_every < 1 || ckpt_every > LDPC_UNROLL_MAX_CKPT_EVERY) return LDPC_EINVAL;
  return (int64_t)((T + ckpt_every - 1) / ckpt_every) * (int64_t)(c->E + c->N);
}

int ldpc_unrolled_forward(const ldpc_code* c, const float* llr, const float* w, const int32_t* trace, int32_t B,
                          int32_t T, int32_t ckpt_every, float* ckpt, float* soft_out, float* c2v_out,
                          void* stream) {
  int dev = 0;
  int rc = unroll_check(c, B, T, ckpt_every, &dev);
  if (rc != LDPC_OK) return rc;
  if (B == 0) return LDPC_OK;
  if (!llr || !w || !soft_out || (T > 0 && !trace)) return LDPC_EINVAL;
  UnrollParams U{};
  unroll_layout(c, ckpt_every, U);
  const int lds_limit = std::min(device_lds_limit(dev), 160 * 1024);
  if (U.lds_fwd > lds_limit) return LDPC_ECAPACITY;
  U.B = B; U.T = T; U.ckpt_every = ckpt_every; U.n_ckpt = (T + ckpt_every - 1) / ckpt_every;
  U.llr = llr; U.w = w; U.trace = trace; U.ckpt = ckpt; U.soft_out = soft_out; U.c2v_out = c2v_out;
  const int per_cu = std::max(1, std::min(32, (160 * 1024) / std::max(U.lds_fwd, 1)));
  const int grid = (int)std::min<long long>(B, (long long)device_cu_count(dev) * per_cu);
  hipError_t he = raise_lds_limit(FAM_UNROLL, lds_limit, set_unroll_lds_limit);
  if (he == hipSuccess) he = launch_unroll_fwd(c->dev, U, grid, (hipStream_t)stream);
  return he == hipSuccess ? LDPC_OK : hip_fail(he);
}

int ldpc_unrolled_backward(const ldpc_code* c, const float* w, const int32_t* trace, int32_t B, int32_t T,
                           int32_t ckpt_every, const float* ckpt, const float* grad_soft, float* grad_llr,
                           float* grad_w, void* stream) {
  int dev = 0;
  int rc = unroll_check(c, B, T, ckpt_every, &dev);
  if (rc != LDPC_OK) return rc;
  if (!grad_w) return LDPC_EINVAL;
  if (B > 0 && (!w || !grad_soft || !grad_llr || (T > 0 && (!trace || !ckpt)))) return LDPC_EINVAL;
  UnrollParams U{};
  unroll_layout(c, ckpt_every, U);
  const int lds_limit = std::min(device_lds_limit(dev), 160 * 1024);
  if (U.lds_bwd > lds_limit) return LDPC_ECAPACITY;
  U.B = B; U.T = T; U.ckpt_every = ckpt_every; U.n_ckpt = (T + ckpt_every - 1) / ckpt_every;
  U.w = w; U.trace = trace; U.ckpt = const_cast<float*>(ckpt); U.grad_soft = grad_soft; U.grad_llr = grad_llr;
  hipStream_t st = (hipStream_t)stream;
  const int nch = std::max(1, std::min(64, (int)B));
  const int chunk = B > 0 ? (B + nch - 1) / nch : 1;
  const size_t part_bytes = (size_t)B * c->E * 4, chunk_bytes = (size_t)nch * c->E * 4;
  void* scratch = nullptr;
  hipError_t he = scratch_alloc(&scratch, part_bytes + chunk_bytes, st);
  if (he != hipSuccess) return he == hipErrorOutOfMemory ? LDPC_ENOMEM : hip_fail(he);
  U.gw_part = reinterpret_cast<float*>(scratch);
  float* chunks = reinterpret_cast<float*>((char*)scratch + part_bytes);
  const int per_cu = std::max(1, std::min(32, (160 * 1024) / std::max(U.lds_bwd, 1)));
  const int grid = (int)std::max<long long>(1, std::min<long long>(B, (long long)device_cu_count(dev) * per_cu));
  he = raise_lds_limit(FAM_UNROLL, lds_limit, set_unroll_lds_limit);
  if (he == hipSuccess) he = launch_unroll_bwd(c->dev, U, grid, chunks, nch, chunk, grad_w, st);
  (void)hipFreeAsync(scratch, st);
  return he == hipSuccess ? LDPC_OK : hip_fail(he);
}

// ------------------------------------------------------------------------------------------
// SNR sweeps captured into a hipGraph
// ------------------------------------------------------------------------------------------
int ldpc_awgn_frames(const uint8_t* codewords, int32_t P, int32_t N, int32_t B, float sigma2, uint64_t seed,
                     int32_t point, float* llr_out, void* stream) {
  if (P < 1 || N < 1 || B < 0 || point < 0 || !(sigma2 > 0.0f) || !std::isfinite(sigma2)) return LDPC_EINVAL;
  if (B == 0) return LDPC_OK;
  if (!codewords || !llr_out) return LDPC_EINVAL;
  hipError_t he = launch_awgn_frames(codewords, P, N, B, sigma2, nullptr, seed, point, llr_out, (hipStream_t)stream);
  return he == hipSuccess ? LDPC_OK : hip_fail(he);
}

}  // extern "C"

struct ldpc_sweep {
  const ldpc_code* code = nullptr;
  int S = 0, B = 0, P = 0;
  float* llr = nullptr;
  uint8_t* bits = nullptr;
  int64_t* upd = nullptr;
  int64_t* counters = nullptr;  // [S][4]
  uint64_t* seed = nullptr;
  void* scratch = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void sweep_release(ldpc_sweep* w) {
  if (!w) return;
  if (w->exec) (void)hipGraphExecDestroy(w->exec);
  if (w->graph) (void)hipGraphDestroy(w->graph);
  if (w->cap) (void)hipStreamDestroy(w->cap);
  for (void* p : {(void*)w->llr, (void*)w->bits, (void*)w->upd, (void*)w->counters, (void*)w->seed, w->scratch})
    if (p) (void)hipFree(p);
  delete w;
}

}  // namespace

extern "C" {

int ldpc_sweep_create(const ldpc_code* c, const ldpc_schedule* s, int64_t max_updates, const uint8_t* codewords,
                      int32_t P, const float* ebn0_db, int32_t S, float rate, int32_t B, ldpc_sweep** out) {
  if (!out) return LDPC_EINVAL;
  *out = nullptr;
  if (!c || !s || !codewords || P < 1 || !ebn0_db || S < 1 || S > 4096 || B < 1 || !(rate > 0.0f && rate <= 1.0f))
    return LDPC_EINVAL;
  if (s->kind == LDPC_REPLAY) return LDPC_EUNSUPPORTED;
  std::vector<float> sigma2(S);
  for (int p = 0; p < S; ++p) {
    if (!std::isfinite(ebn0_db[p])) return LDPC_EINVAL;
    sigma2[p] = (float)(1.0 / (2.0 * rate * std::pow(10.0, ebn0_db[p] / 10.0)));
  }
  ldpc_sweep* w = new (std::nothrow) ldpc_sweep();
  if (!w) return LDPC_ENOMEM;
  w->code = c;
  w->S = S;
  w->B = B;
  w->P = P;
  hipError_t he = hipMalloc((void**)&w->llr, (size_t)B * c->N * sizeof(float));
  if (he == hipSuccess) he = hipMalloc((void**)&w->bits, (size_t)B * c->N);
  if (he == hipSuccess) he = hipMalloc((void**)&w->upd, (size_t)B * sizeof(int64_t));
  if (he == hipSuccess) he = hipMalloc((void**)&w->counters, (size_t)S * 4 * sizeof(int64_t));
  if (he == hipSuccess) he = hipMalloc((void**)&w->seed, sizeof(uint64_t));
  if (he != hipSuccess) {
    sweep_release(w);
    return he == hipErrorOutOfMemory ? LDPC_ENOMEM : hip_fail(he);
  }
  ldpc_outputs o{};
  o.bits = w->bits;
  o.updates_used = w->upd;
  ldpc_tuning t{};
  const bool tuned = lookup_tuning(c, s->kind, s->arith, t);
  DecodePlan pl;
  int rc = plan_decode(c, s, w->llr, B, max_updates, nullptr, 0, &o, tuned ? &t : nullptr, pl);
  if (rc != LDPC_OK) {
    sweep_release(w);
    return rc;
  }
  if (pl.scratch_bytes && (he = hipMalloc(&w->scratch, pl.scratch_bytes)) != hipSuccess) {
    sweep_release(w);
    return he == hipErrorOutOfMemory ? LDPC_ENOMEM : hip_fail(he);
  }
  if ((he = plan_lds_limits(pl)) == hipSuccess) he = hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking);
  // graph: zero the counters, then per point generate -> decode -> count
  if (he == hipSuccess) he = hipStreamBeginCapture(w->cap, hipStreamCaptureModeRelaxed);
  if (he == hipSuccess) {
    hipError_t ce = launch_fill_u64(w->counters, 4 * S, 0, w->cap);
    for (int p = 0; p < S && ce == hipSuccess; ++p) {
      ce = launch_awgn_frames(codewords, P, c->N, B, sigma2[p], w->seed, 0, p, w->llr, w->cap);
      if (ce == hipSuccess) ce = enqueue_decode(c, pl, w->scratch, w->cap, false);
      if (ce == hipSuccess) ce = launch_count_errors(w->bits, codewords, P, c->N, B, w->upd, w->counters + 4 * p, w->cap);
    }
    he = hipStreamEndCapture(w->cap, &w->graph);
    if (ce != hipSuccess) he = ce;
  }
  if (he == hipSuccess) he = hipGraphInstantiate(&w->exec, w->graph, nullptr, nullptr, 0);
  if (he != hipSuccess) {
    sweep_release(w);
    return hip_fail(he);
  }
  *out = w;
  return LDPC_OK;
}

int ldpc_sweep_run(ldpc_sweep* w, uint64_t seed, int64_t* counters, void* stream) {
  if (!w || !counters) return LDPC_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t he = launch_fill_u64(reinterpret_cast<int64_t*>(w->seed), 1, seed, st);
  if (he == hipSuccess) he = hipGraphLaunch(w->exec, st);
  if (he == hipSuccess)
    he = hipMemcpyAsync(counters, w->counters, (size_t)w->S * 4 * sizeof(int64_t), hipMemcpyDeviceToDevice, st);
  return he == hipSuccess ? LDPC_OK : hip_fail(he);
}

void ldpc_sweep_free(ldpc_sweep* w) {
  if (!w) return;
  (void)hipDeviceSynchronize();
  sweep_release(w);
}

}  // extern "C"
