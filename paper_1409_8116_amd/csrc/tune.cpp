// Kernel-shape autotuner: for one line pass, time every kernel shape that can
// hold it and keep the fastest.  Results are kept per process and, when the
// environment variable MPOIS_TUNE_CACHE names a file, in that file as lines
//   <device name> <key> <shape id>
// so later processes reuse them.  A line for another device, or one that names
// a shape that cannot hold the pass, is ignored.
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

namespace mpois {
int num_kernel_cfgs();
void kernel_cfg(int i, int* f64, int* np, int* nt, int* pmax);
int kernel_cfg_rader(int i);
int kernel_cfg_slim(int i);
size_t line_pass_lds(int cfg, int n, int P);
hipError_t launch_line_pass(int cfg, const PassArgs& a, hipStream_t s);

bool tune_enabled(unsigned flags) { return (flags & MPOIS_FLAG_TUNE) != 0; }

namespace {

std::mutex g_mu;
std::map<std::string, int> g_cache;
bool g_loaded = false;

std::string device_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string s = prop.gcnArchName;
  for (auto& c : s)
    if (c == ' ') c = '_';
  return s + "_cu" + std::to_string(prop.multiProcessorCount);
}

void load_file() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("MPOIS_TUNE_CACHE");
  if (!path) return;
  std::ifstream in(path);
  const std::string dev = device_name();
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ss(line);
    std::string d, key;
    int cfg = -1;
    if (ss >> d >> key >> cfg && d == dev && cfg >= 0 && cfg < num_kernel_cfgs()) g_cache[key] = cfg;
  }
}

void save_entry(const std::string& key, int cfg) {
  const char* path = std::getenv("MPOIS_TUNE_CACHE");
  if (!path) return;
  std::ofstream out(path, std::ios::app);
  if (out) out << device_name() << " " << key << " " << cfg << "\n";
}

bool fits(int cfg, bool f64, int n, int P, bool rader, bool odd) {
  int cf64, np, nt, pmax;
  kernel_cfg(cfg, &cf64, &np, &nt, &pmax);
  if ((cf64 != 0) != f64 || P > pmax) return false;
  if (rader && !kernel_cfg_rader(cfg)) return false;
  if (odd && kernel_cfg_slim(cfg)) return false;
  return line_pass_lds(cfg, n, P) <= size_t(160 * 1024);
}

}  // namespace

int tune_pass(const PassArgs& proto, int fallback, bool f64, bool rader, bool odd) {
  const int n = proto.ax.n, P = proto.ax.P;
  std::ostringstream k;
  k << (f64 ? "f64" : "f32") << "/kf" << proto.kind_f << "/kb" << proto.kind_b << "/n" << n << "/P" << P << "/lines"
    << proto.nlines << "/inner" << proto.inner;
  const std::string key = k.str();
  std::lock_guard<std::mutex> lock(g_mu);
  load_file();
  auto it = g_cache.find(key);
  if (it != g_cache.end() && fits(it->second, f64, n, P, rader, odd)) return it->second;

  std::vector<int> cands;
  for (int i = 0; i < num_kernel_cfgs(); ++i)
    if (fits(i, f64, n, P, rader, odd)) cands.push_back(i);
  if (cands.size() <= 1) return cands.empty() ? fallback : cands[0];

  // scratch arrays of the pass's own size (values do not affect the timing)
  const size_t elems = size_t(proto.nlines) * size_t(n);
  const size_t es = f64 ? 8 : 4;
  void *src = nullptr, *dst = nullptr;
  double* shift = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = fallback;
  if (hipMalloc(&src, elems * es) == hipSuccess && hipMalloc(&dst, elems * es) == hipSuccess &&
      hipMalloc(reinterpret_cast<void**>(&shift), 64) == hipSuccess &&
      hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
      hipEventCreate(&e1) == hipSuccess && hipMemsetAsync(src, 0, elems * es, s) == hipSuccess &&
      hipMemsetAsync(shift, 0, 64, s) == hipSuccess) {
    PassArgs a = proto;
    a.src = src;
    a.dst = dst;
    a.src_f64 = f64 ? 1 : 0;
    a.dst_f64 = f64 ? 1 : 0;
    a.update = 0;
    a.shift = shift;
    float best_ms = 1e30f;
    for (int cfg : cands) {
      bool ok = launch_line_pass(cfg, a, s) == hipSuccess;  // warm-up
      ok = ok && hipEventRecord(e0, s) == hipSuccess;
      for (int r = 0; r < 3 && ok; ++r) ok = launch_line_pass(cfg, a, s) == hipSuccess;
      ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
      float ms = 0.f;
      if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best_ms) {
        best_ms = ms;
        best = cfg;
      }
    }
    if (std::getenv("MPOIS_LOG")) std::fprintf(stderr, "[mpois tune] %s -> shape %d (%.3f ms)\n", key.c_str(), best,
                                               best_ms / 3);
  }
  (void)hipGetLastError();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  if (shift) (void)hipFree(shift);
  g_cache[key] = best;
  save_entry(key, best);
  return best;
}

}  // namespace mpois
