// Autotuner measurements and decision cache.  The plan layer enumerates the
// candidates of a line pass (kernel shapes that can hold it, and alternative
// radix plans of its DFT length: other stage orders and splits, a Bluestein
// convolution instead of a Rader stage or a large odd radix), times each with
// tune_time on scratch arrays, and keeps the fastest.
#include "tune.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "mpois.h"

#ifndef MPOIS_BUILD_ID
#define MPOIS_BUILD_ID "dev"
#endif

namespace mpois {
hipError_t launch_line_pass(int cfg, const PassArgs& a, hipStream_t s);
hipError_t launch_line_pass_batch(int cfg, const BatchPassArgs& b, int blocks, size_t lds, hipStream_t s);
size_t line_pass_lds(int cfg, int n, int P);
void kernel_cfg(int i, int* f64, int* np, int* nt, int* pmax);

bool tune_enabled(unsigned flags) { return (flags & MPOIS_FLAG_TUNE) != 0; }

struct TuneSession {
  void* src = nullptr;
  void* dst = nullptr;
  size_t bytes = 0;
  double* shift = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = false;
  // the batch kernel's tables for a one-grid batch: its pass description,
  // block -> (grid 0, tile b) maps of up to kMaxBlocks blocks, pointer tables
  PassArgs* args = nullptr;
  int* prob = nullptr;
  int* idx = nullptr;
  void** tabs = nullptr;  // src, dst
};

constexpr int kMaxTuneBlocks = 1 << 16;

TuneSession* tune_begin() {
  TuneSession* t = new TuneSession();
  t->ok = hipStreamCreateWithFlags(&t->s, hipStreamNonBlocking) == hipSuccess &&
          hipEventCreate(&t->e0) == hipSuccess && hipEventCreate(&t->e1) == hipSuccess &&
          hipMalloc(reinterpret_cast<void**>(&t->shift), 64) == hipSuccess &&
          hipMemsetAsync(t->shift, 0, 64, t->s) == hipSuccess;
  if (t->ok) {
    std::vector<int> idx(kMaxTuneBlocks);
    for (int i = 0; i < kMaxTuneBlocks; ++i) idx[i] = i;
    t->ok = hipMalloc(reinterpret_cast<void**>(&t->args), sizeof(PassArgs)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&t->prob), kMaxTuneBlocks * sizeof(int)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&t->idx), kMaxTuneBlocks * sizeof(int)) == hipSuccess &&
            hipMalloc(reinterpret_cast<void**>(&t->tabs), 2 * sizeof(void*)) == hipSuccess &&
            hipMemsetAsync(t->prob, 0, kMaxTuneBlocks * sizeof(int), t->s) == hipSuccess &&
            hipMemcpyAsync(t->idx, idx.data(), kMaxTuneBlocks * sizeof(int), hipMemcpyHostToDevice, t->s) ==
                hipSuccess &&
            hipStreamSynchronize(t->s) == hipSuccess;
  }
  if (!t->ok) (void)hipGetLastError();
  return t;
}

void tune_end(TuneSession* t) {
  if (!t) return;
  if (t->s) (void)hipStreamSynchronize(t->s);
  if (t->src) (void)hipFree(t->src);
  if (t->dst) (void)hipFree(t->dst);
  if (t->shift) (void)hipFree(t->shift);
  for (void* p : {static_cast<void*>(t->args), static_cast<void*>(t->prob), static_cast<void*>(t->idx),
                  static_cast<void*>(t->tabs)})
    if (p) (void)hipFree(p);
  if (t->e0) (void)hipEventDestroy(t->e0);
  if (t->e1) (void)hipEventDestroy(t->e1);
  if (t->s) (void)hipStreamDestroy(t->s);
  (void)hipGetLastError();
  delete t;
}

// Scratch of at least `bytes` per array, zero-filled (grown, never shrunk,
// within a session).
static bool ensure_scratch(TuneSession* t, size_t bytes) {
  if (bytes <= t->bytes) return true;
  (void)hipStreamSynchronize(t->s);
  if (t->src) (void)hipFree(t->src);
  if (t->dst) (void)hipFree(t->dst);
  t->src = t->dst = nullptr;
  t->bytes = 0;
  if (hipMalloc(&t->src, bytes) != hipSuccess || hipMalloc(&t->dst, bytes) != hipSuccess ||
      hipMemsetAsync(t->src, 0, bytes, t->s) != hipSuccess || hipMemsetAsync(t->dst, 0, bytes, t->s) != hipSuccess) {
    (void)hipGetLastError();
    if (t->src) (void)hipFree(t->src);
    if (t->dst) (void)hipFree(t->dst);
    t->src = t->dst = nullptr;
    return false;
  }
  t->bytes = bytes;
  return true;
}

double tune_time_batch(TuneSession* t, const PassArgs& proto, int cfg, int64_t lines) {
  if (!t || !t->ok) return -1.0;
  int cf64, np, nt, pmax;
  kernel_cfg(cfg, &cf64, &np, &nt, &pmax);
  const int64_t blocks = (lines + 2 * np - 1) / (2 * np);
  if (blocks > kMaxTuneBlocks) return -1.0;
  if (!ensure_scratch(t, size_t(lines) * size_t(proto.ax.n) * 8)) return -1.0;
  PassArgs a = proto;
  a.nlines = lines;
  if (a.inner > 1 && lines % a.inner != 0) a.inner = 1;
  a.lam_a = nullptr;
  a.lam_b = nullptr;
  a.src_vnb = a.dst_vnb = a.inner;
  a.src_va = a.dst_va = int64_t(a.ax.n) * a.inner;
  a.src_vb = a.dst_vb = 1;
  a.src_vd = a.dst_vd = a.inner;
  a.contig = 1;
  void* tabs[2] = {t->src, t->dst};
  if (hipMemcpyAsync(t->args, &a, sizeof(a), hipMemcpyHostToDevice, t->s) != hipSuccess ||
      hipMemcpyAsync(t->tabs, tabs, sizeof(tabs), hipMemcpyHostToDevice, t->s) != hipSuccess ||
      hipStreamSynchronize(t->s) != hipSuccess) {
    (void)hipGetLastError();
    return -1.0;
  }
  BatchPassArgs b{};
  b.args = t->args;
  b.tile_prob = t->prob;
  b.tile_idx = t->idx;
  b.src_tab = t->tabs;
  b.dst_tab = t->tabs + 1;
  b.src_f64 = proto.src_f64;
  b.dst_f64 = proto.dst_f64;
  const size_t lds = line_pass_lds(cfg, proto.ax.n, proto.ax.P);
  bool ok = launch_line_pass_batch(cfg, b, int(blocks), lds, t->s) == hipSuccess;  // warm-up
  ok = ok && hipEventRecord(t->e0, t->s) == hipSuccess;
  constexpr int kReps = 3;
  for (int r = 0; r < kReps && ok; ++r) ok = launch_line_pass_batch(cfg, b, int(blocks), lds, t->s) == hipSuccess;
  ok = ok && hipEventRecord(t->e1, t->s) == hipSuccess && hipEventSynchronize(t->e1) == hipSuccess;
  float ms = 0.f;
  if (!ok || hipEventElapsedTime(&ms, t->e0, t->e1) != hipSuccess) {
    (void)hipGetLastError();
    return -1.0;
  }
  return double(ms) / kReps;
}

double tune_time(TuneSession* t, const PassArgs& proto, int cfg, int64_t lines) {
  if (!t || !t->ok) return -1.0;
  const size_t es = 8;  // scratch sized for double, valid for either element type
  const int64_t nl = lines > 0 ? lines : proto.nlines;
  if (!ensure_scratch(t, size_t(nl) * size_t(proto.ax.n) * es)) return -1.0;
  PassArgs a = proto;
  a.nlines = nl;
  // a pass over nl lines of a (nl / inner, n, inner) box keeps its stride class
  if (a.inner > 1 && nl % a.inner != 0) a.inner = 1;
  a.src = t->src;
  a.dst = t->dst;
  a.update = 0;
  a.shift = t->shift;
  a.lam_a = nullptr;  // eigenvalue tables of the other axes belong to the real box
  a.lam_b = nullptr;
  bool ok = launch_line_pass(cfg, a, t->s) == hipSuccess;  // warm-up
  ok = ok && hipEventRecord(t->e0, t->s) == hipSuccess;
  constexpr int kReps = 3;
  for (int r = 0; r < kReps && ok; ++r) ok = launch_line_pass(cfg, a, t->s) == hipSuccess;
  ok = ok && hipEventRecord(t->e1, t->s) == hipSuccess && hipEventSynchronize(t->e1) == hipSuccess;
  float ms = 0.f;
  if (!ok || hipEventElapsedTime(&ms, t->e0, t->e1) != hipSuccess) {
    (void)hipGetLastError();
    return -1.0;
  }
  return double(ms) / kReps;
}

namespace {

std::mutex g_mu;
std::map<std::string, std::pair<int, int>> g_cache;
bool g_loaded = false;

std::string device_key() {
  int dev = 0, rt = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  (void)hipRuntimeGetVersion(&rt);
  std::string s = prop.gcnArchName;
  for (auto& c : s)
    if (c == ' ' || c == ':') c = '_';
  return s + "_cu" + std::to_string(prop.multiProcessorCount) + "_hip" + std::to_string(rt) + "_" + MPOIS_BUILD_ID;
}

void load_file() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("MPOIS_TUNE_CACHE");
  if (!path) return;
  std::ifstream in(path);
  const std::string dev = device_key();
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ss(line);
    std::string d, key;
    int a = -1, b = -1;
    if (ss >> d >> key >> a >> b && d == dev) g_cache[key] = {a, b};
  }
}

}  // namespace

bool tune_lookup(const std::string& key, int* a, int* b) {
  std::lock_guard<std::mutex> lock(g_mu);
  load_file();
  auto it = g_cache.find(key);
  if (it == g_cache.end()) return false;
  *a = it->second.first;
  *b = it->second.second;
  return true;
}

void tune_store(const std::string& key, int a, int b) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_cache[key] = {a, b};
  const char* path = std::getenv("MPOIS_TUNE_CACHE");
  if (!path) return;
  std::ofstream out(path, std::ios::app);
  if (out) out << device_key() << " " << key << " " << a << " " << b << "\n";
}

}  // namespace mpois
