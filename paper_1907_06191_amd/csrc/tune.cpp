// Launch-shape autotuner of the stage kernels.
#include "tune.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <sstream>
#include <vector>

namespace dgd {
namespace {

std::mutex g_mu;
std::map<std::string, TuneParams> g_table;

struct DeviceInfo {
  std::string arch;
  int cus = 0;
};

DeviceInfo device_info() {
  int dev = 0;
  DGD_HIP_CHECK(hipGetDevice(&dev));
  static std::mutex mu;
  static std::map<int, DeviceInfo> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  hipDeviceProp_t prop;
  DGD_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
  DeviceInfo d;
  d.arch = prop.gcnArchName;
  const size_t colon = d.arch.find(':');
  if (colon != std::string::npos) d.arch.resize(colon);
  DGD_HIP_CHECK(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
  cache[dev] = d;
  return d;
}

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  Events() {
    DGD_HIP_CHECK(hipEventCreate(&a));
    DGD_HIP_CHECK(hipEventCreate(&b));
  }
  ~Events() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

// DGD_TUNE_CACHE names a file holding the shape table in the text form of
// tune_export: read once before the first lookup (a missing or malformed
// file is ignored) and rewritten after every newly tuned key.
const char* cache_path() {
  const char* p = std::getenv("DGD_TUNE_CACHE");
  return p && *p ? p : nullptr;
}

void load_cache_once();

bool valid(const TuneParams& p) {
  return (p.epw == 1 || p.epw == 2 || p.epw == 4 || p.epw == 8) &&
         (p.waves == 1 || p.waves == 2 || p.waves == 4) && (p.remap == 0 || p.remap == 1) &&
         p.grid_per_cu >= 0 && p.grid_per_cu <= 64;
}

}  // namespace

std::string tune_key(int np, int prec, const char* kernel, int R, int64_t E) {
  const int e2 = E > 0 ? (int)std::floor(std::log2((double)E)) : 0;
  std::ostringstream k;
  k << device_info().arch << "|np" << np << "|" << (prec == DGD_FP64 ? "fp64" : "fp32") << "|"
    << kernel << "|R" << R << "|E2^" << e2;
  return k.str();
}

bool tune_find(const std::string& key, TuneParams* out) {
  load_cache_once();
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(key);
  if (it == g_table.end()) return false;
  *out = it->second;
  return true;
}

Shape tune_shape(const TuneParams& p, int64_t units) {
  const int64_t grid = p.grid_per_cu > 0 ? (int64_t)p.grid_per_cu * device_info().cus : 0;
  return element_shape(units, p.epw, p.waves, p.remap != 0, grid);
}

TuneParams tune_stage(const std::string& key, int64_t units, int prec, int64_t n_values, void* a,
                      void* b, const void* base, const StageLaunch& launch_one, hipStream_t st) {
  const int64_t n = n_values;
  if (prec == DGD_FP64)
    launch_fill_random((double*)a, n, 0x5eedull, st);
  else
    launch_fill_random_f32((float*)a, n, 0x5eedull, st);
  DGD_HIP_CHECK(hipGetLastError());
  if (!base) base = a;
  // One timed unit is an SSP-RK3 step's pattern of launches: a stage
  // without a base state (a -> b), then two stages reading `base`
  // (b -> a, a -> b), so the tuned shape is the fastest for the mix of
  // kernels a step runs, not for one of them.
  auto step = [&](const Shape& sh) {
    launch_one(sh, a, nullptr, b);
    launch_one(sh, b, base, a);
    launch_one(sh, a, base, b);
  };
  Events ev;
  // ms per launch over `reps` steps, after one untimed step
  auto time_ms = [&](const TuneParams& p, int reps) {
    const Shape sh = tune_shape(p, units);
    step(sh);
    DGD_HIP_CHECK(hipEventRecord(ev.a, st));
    for (int i = 0; i < reps; ++i) step(sh);
    DGD_HIP_CHECK(hipEventRecord(ev.b, st));
    DGD_HIP_CHECK(hipEventSynchronize(ev.b));
    DGD_HIP_CHECK(hipGetLastError());
    float ms = 0;
    DGD_HIP_CHECK(hipEventElapsedTime(&ms, ev.a, ev.b));
    return (double)ms / (3.0 * reps);
  };

  std::vector<TuneParams> cand;
  for (int epw : {1, 2, 4}) {
    for (int waves : {1, 2, 4})
      for (int remap : {0, 1})
        for (int gpc : {0, 4, 8, 16}) {
          TuneParams p;
          p.epw = epw;
          p.waves = waves;
          p.remap = remap;
          p.grid_per_cu = gpc;
          cand.push_back(p);
        }
  }
  // Warm the device up (clocks ramp up under load: a cold start would
  // favour whatever is timed last) for about 30 ms; time every candidate
  // for about 3 ms twice, in forward and in reverse order, keeping the
  // better time; then time the best six again in three interleaved rounds
  // of about 10 ms each and keep each one's best.
  double est = time_ms(TuneParams(), 1);
  for (double spent = 0; spent < 30.0;) {
    const int n = std::max(1, std::min(100, (int)std::ceil(10.0 / std::max(3.0 * est, 1e-3))));
    est = time_ms(TuneParams(), n);
    spent += std::max(3.0 * est, 1e-3) * (n + 1);
  }
  auto reps_for = [&](double ms_target) {
    return std::max(1, std::min(300, (int)std::ceil(ms_target / std::max(3.0 * est, 1e-3))));
  };
  const int reps = reps_for(3.0);
  for (auto& p : cand) p.ms = time_ms(p, reps);
  for (auto it = cand.rbegin(); it != cand.rend(); ++it) it->ms = std::min(it->ms, time_ms(*it, reps));
  std::sort(cand.begin(), cand.end(),
            [](const TuneParams& x, const TuneParams& y) { return x.ms < y.ms; });
  const size_t top = std::min<size_t>(6, cand.size());
  const int reps_fine = reps_for(10.0);
  for (int round = 0; round < 3; ++round)
    for (size_t i = 0; i < top; ++i) {
      const double t = time_ms(cand[i], reps_fine);
      cand[i].ms = round == 0 ? t : std::min(cand[i].ms, t);
    }
  std::sort(cand.begin(), cand.begin() + top,
            [](const TuneParams& x, const TuneParams& y) { return x.ms < y.ms; });
  const TuneParams best = cand[0];
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[key] = best;
  }
  if (const char* path = cache_path()) {
    const std::string text = tune_export();
    const std::string tmp = std::string(path) + ".tmp";
    if (std::FILE* f = std::fopen(tmp.c_str(), "w")) {
      const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
      if (std::fclose(f) == 0 && ok) std::rename(tmp.c_str(), path);
    }
  }
  return best;
}

std::string tune_export() {
  std::lock_guard<std::mutex> lk(g_mu);
  std::ostringstream o;
  o.precision(6);
  for (const auto& kv : g_table)
    o << kv.first << ' ' << kv.second.epw << ' ' << kv.second.waves << ' ' << kv.second.remap << ' '
      << kv.second.grid_per_cu << ' ' << kv.second.ms << '\n';
  return o.str();
}

int tune_import(const std::string& text) {
  std::istringstream in(text);
  std::string line;
  std::vector<std::pair<std::string, TuneParams>> rows;
  while (std::getline(in, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ls(line);
    std::string key;
    TuneParams p;
    if (!(ls >> key >> p.epw >> p.waves >> p.remap >> p.grid_per_cu >> p.ms) || !valid(p))
      throw Error{DGD_EINVAL, "bad tuning table line: " + line};
    rows.emplace_back(key, p);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& r : rows) g_table[r.first] = r.second;
  return (int)rows.size();
}

namespace {
void load_cache_once() {
  static std::once_flag once;
  std::call_once(once, [] {
    const char* path = cache_path();
    if (!path) return;
    std::FILE* f = std::fopen(path, "r");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    std::fclose(f);
    try {
      tune_import(text);
    } catch (const Error&) {
      // a malformed cache is ignored: the shapes are tuned again
    }
  });
}
}  // namespace

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
}

}  // namespace dgd
