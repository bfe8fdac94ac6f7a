// Launch-shape autotuner for the hop kernel, with a small JSON cache file.
//
// The paper measures the operator over several SIMD tile shapes and finds
// little difference (Sec. 3); on gfx950 the equivalent knobs are the workgroup
// size, whether blocks are mapped so that each XCD works on one contiguous
// slab of the lattice (its own L2), and whether the links (read once) are
// loaded non-temporally, and whether one lane or a quad of lanes (one lattice
// direction each) computes an output site. The tuner times each candidate with HIP
// events on scratch fields and keeps the fastest per (lattice, precision).
//
// Cache format: one JSON object, keys "Lx.Ly.Lz.Lt:prec", values
// {"block": B, "remap": R, "nt": N, "split": S, "us": T}. The path comes from lqcd_autotune's
// argument or from the LQCD_TUNE_CACHE environment variable. Other tuners
// (the batched hop) keep their entries in the same file under their own keys
// through tune_cache_get / tune_cache_put, the four numbers in the same fields.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "internal.h"
#include "ops.h"
#include "tune.h"

namespace lq {

namespace {

std::string key_of(const lqcd_ctx* c, int prec) {
  std::ostringstream o;
  o << c->g.lx << "." << c->g.ly << "." << c->g.lz << "." << c->g.lt << ":" << prec;
  return o.str();
}

struct Entry {
  int block = 256, remap = 1, nt = 0, split = 1;
  double us = 0;
};

// Minimal reader for the flat format written below.
std::map<std::string, Entry> read_cache(const std::string& path) {
  std::map<std::string, Entry> m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t pos = 0;
  while ((pos = s.find('"', pos)) != std::string::npos) {
    const size_t end = s.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = s.substr(pos + 1, end - pos - 1);
    const size_t ob = s.find('{', end), cb = s.find('}', end);
    if (ob == std::string::npos || cb == std::string::npos || key.find(':') == std::string::npos) {
      pos = end + 1;
      continue;
    }
    const std::string body = s.substr(ob, cb - ob);
    Entry e;
    auto num = [&](const char* name, double& out) {
      const size_t k = body.find(std::string("\"") + name + "\"");
      if (k == std::string::npos) return;
      const size_t colon = body.find(':', k);
      if (colon != std::string::npos) out = std::atof(body.c_str() + colon + 1);
    };
    double b = 256, r = 1, nt = 0, sp = 1, us = 0;
    num("block", b);
    num("remap", r);
    num("nt", nt);
    num("split", sp);
    e.split = (int)sp;
    num("us", us);
    e.block = (int)b;
    e.remap = (int)r;
    e.nt = (int)nt;
    e.us = us;
    m[key] = e;
    pos = cb + 1;
  }
  return m;
}

bool write_cache(const std::string& path, const std::map<std::string, Entry>& m) {
  std::ofstream f(path);
  if (!f) return false;
  f << "{\n";
  size_t n = 0;
  for (const auto& kv : m) {
    f << "  \"" << kv.first << "\": {\"block\": " << kv.second.block << ", \"remap\": " << kv.second.remap
      << ", \"nt\": " << kv.second.nt << ", \"split\": " << kv.second.split << ", \"us\": " << kv.second.us << "}" << (++n < m.size() ? "," : "") << "\n";
  }
  f << "}\n";
  return true;
}

bool valid(const Entry& e) {
  return (e.block == 64 || e.block == 128 || e.block == 192 || e.block == 256) && e.remap >= 0 && e.remap <= 2 &&
         (e.nt == 0 || e.nt == 1) && (e.split == 1 || e.split == 2 || e.split == 4);
}

bool valid_for(const lqcd_ctx* c, int prec, const Entry& e) {
  if (e.split == 0) return (e.nt == 0 || e.nt == 1) && march_shape_ok(c->g, prec, e.block, e.remap);
  if (!valid(e)) return false;
  return e.remap != 2 || c->g.lz % 8 == 0;
}

}  // namespace

bool tune_cache_get(const std::string& key, int v[4]) {
  const char* env = std::getenv("LQCD_TUNE_CACHE");
  if (!env || !*env) return false;
  const auto m = read_cache(env);
  auto it = m.find(key);
  if (it == m.end()) return false;
  v[0] = it->second.block;
  v[1] = it->second.split;
  v[2] = it->second.remap;
  v[3] = it->second.nt;
  return true;
}

int tune_cache_put(const std::string& key, const int v[4], double us) {
  const char* env = std::getenv("LQCD_TUNE_CACHE");
  if (!env || !*env) return LQCD_OK;
  auto m = read_cache(env);
  Entry e;
  e.block = v[0];
  e.split = v[1];
  e.remap = v[2];
  e.nt = v[3];
  e.us = us;
  m[key] = e;
  if (!write_cache(env, m)) return set_error(LQCD_EINVAL, std::string("cannot write tune cache ") + env);
  return LQCD_OK;
}

int tune_load_defaults(lqcd_ctx* c) {
  const char* env = std::getenv("LQCD_TUNE_CACHE");
  if (!env || !*env) return LQCD_OK;
  const auto m = read_cache(env);
  for (int p = 0; p < 3; ++p) {
    auto it = m.find(key_of(c, p));
    if (it != m.end() && valid_for(c, p, it->second)) {
      c->hop_block[p] = it->second.block;
      c->hop_remap[p] = it->second.remap;
      c->hop_nt[p] = it->second.nt;
      c->hop_split[p] = it->second.split;
    }
  }
  return LQCD_OK;
}

}  // namespace lq

using namespace lq;

extern "C" int lqcd_autotune(lqcd_ctx* c, int prec, const char* path) {
  if (!c) return set_error(LQCD_EINVAL, "null argument");
  if (prec < 0 || prec > 2) return set_error(LQCD_EINVAL, "bad precision");
  if (!c->have_gauge || !c->have_clover) return set_error(LQCD_ESTATE, "set_gauge and set_clover must come first");
  // three input/output pairs in rotation, so that the timed launches stream
  // from HBM instead of hitting in the Infinity Cache as a solver's would not
  const size_t bytes = spinor_bytes(prec, c->g.vh);
  constexpr int NB = 3;
  void* buf[2 * NB] = {};
  for (int k = 0; k < 2 * NB; ++k) {
    if (hipMalloc(&buf[k], bytes) != hipSuccess) {
      for (int j = 0; j < k; ++j) (void)hipFree(buf[j]);
      (void)hipGetLastError();
      return set_error(LQCD_ENOMEM, "autotune scratch allocation failed");
    }
    (void)hipMemsetAsync(buf[k], 0, bytes, c->stream);
  }
  const bool verbose = std::getenv("LQCD_TUNE_VERBOSE") != nullptr;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int blocks[] = {64, 128, 192, 256};
  Entry best;
  best.us = 1e30;
  const int save_b = c->hop_block[prec], save_r = c->hop_remap[prec], save_nt = c->hop_nt[prec],
            save_s = c->hop_split[prec];
  // candidates: the site-parallel kernels (split 1, 2, 4 x block x XCD mapping x
  // non-temporal links) and the plane march (rows per tile x z planes per block)
  std::vector<Entry> cand;
  for (int split : {1, 2, 4})
    for (int nt = 0; nt < 2; ++nt)
      for (int remap = 0; remap < 3; ++remap)
        for (int b : blocks) {
          Entry e;
          e.block = b;
          e.split = split;
          e.remap = remap;
          e.nt = nt;
          if (valid_for(c, prec, e)) cand.push_back(e);
        }
  for (int rows = c->g.ly; rows >= 2; rows /= 2)
    for (int zc : {2, 4, 8}) {
      Entry e;
      e.block = rows * c->g.lxh;
      e.split = 0;
      e.remap = zc;
      e.nt = 1;
      if (e.block >= 64 && valid_for(c, prec, e)) cand.push_back(e);
    }
  int status = LQCD_OK;
  for (const Entry& e : cand) {
      if (status != LQCD_OK) break;
      const int b = e.block, remap = e.remap, nt = e.nt, split = e.split;
      c->hop_block[prec] = b;
      c->hop_remap[prec] = remap;
      c->hop_nt[prec] = nt;
      c->hop_split[prec] = split;
      for (int w = 0; w < 3 && status == LQCD_OK; ++w) status = op_hop(c, prec, 0, buf[w], buf[NB + w], 1.0);
      (void)hipEventRecord(e0, c->stream);
      const int reps = 24;
      for (int r = 0; r < reps && status == LQCD_OK; ++r) status = op_hop(c, prec, 0, buf[r % NB], buf[NB + r % NB], 1.0);
      (void)hipEventRecord(e1, c->stream);
      (void)hipEventSynchronize(e1);
      if (status != LQCD_OK) break;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double us = 1000.0 * ms / reps;
      if (verbose)
        std::fprintf(stderr, "[lqcd tune] %s split %d block %d remap %d nt %d: %.2f us\n", key_of(c, prec).c_str(),
                     split, b, remap, nt, us);
      if (us < best.us) {
        best.us = us;
        best.block = b;
        best.remap = remap;
        best.nt = nt;
        best.split = split;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (void* p : buf) (void)hipFree(p);
  if (status != LQCD_OK) {
    c->hop_block[prec] = save_b;
    c->hop_remap[prec] = save_r;
    c->hop_nt[prec] = save_nt;
    c->hop_split[prec] = save_s;
    return status;
  }
  c->hop_block[prec] = best.block;
  c->hop_remap[prec] = best.remap;
  c->hop_nt[prec] = best.nt;
  c->hop_split[prec] = best.split;
  std::string p = path ? path : "";
  if (p.empty()) {
    const char* env = std::getenv("LQCD_TUNE_CACHE");
    if (env) p = env;
  }
  if (!p.empty()) {
    auto m = read_cache(p);
    m[key_of(c, prec)] = best;
    if (!write_cache(p, m)) return set_error(LQCD_EINVAL, "cannot write tune cache " + p);
  }
  return LQCD_OK;
}

namespace lq {
namespace {

// Read-only stream: every 16-byte word once, summed; the sum is stored only
// if it equals -1, which a zeroed buffer never gives, so the loads stay.
__global__ void __launch_bounds__(256) k_read_probe(const float4* __restrict__ a, size_t n, float* sink) {
  float acc = 0.f;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float4 v = a[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  if (acc == -1.f) sink[0] = acc;
}

__global__ void __launch_bounds__(256) k_copy_probe(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) b[i] = a[i];
}

}  // namespace
}  // namespace lq

extern "C" int lqcd_bandwidth_probe(lqcd_ctx* c, int kind, size_t bytes, int reps, double* gbs) {
  if (!c || !gbs) return set_error(LQCD_EINVAL, "null argument");
  if (kind < 0 || kind > 1 || reps < 1 || bytes < ((size_t)1 << 20))
    return set_error(LQCD_EINVAL, "bandwidth probe: kind 0 or 1, reps >= 1, at least 1 MiB");
  const size_t n = bytes / 16;
  void* a = nullptr;
  void* b = nullptr;
  if (hipMalloc(&a, n * 16) != hipSuccess || hipMalloc(&b, kind == 1 ? n * 16 : 256) != hipSuccess) {
    if (a) (void)hipFree(a);
    (void)hipGetLastError();
    return set_error(LQCD_ENOMEM, "bandwidth probe allocation failed");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int st = LQCD_OK;
  if (hipMemsetAsync(a, 0, n * 16, c->stream) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    st = set_error(LQCD_EHIP, "bandwidth probe set-up failed");
  float best = 1e30f;
  for (int r = 0; r <= reps && st == LQCD_OK; ++r) {  // the first launch is a warm-up
    (void)hipEventRecord(e0, c->stream);
    if (kind == 0)
      hipLaunchKernelGGL(k_read_probe, dim3(2048), dim3(256), 0, c->stream, static_cast<const float4*>(a), n,
                         static_cast<float*>(b));
    else
      hipLaunchKernelGGL(k_copy_probe, dim3(2048), dim3(256), 0, c->stream, static_cast<const float4*>(a),
                         static_cast<float4*>(b), n);
    (void)hipEventRecord(e1, c->stream);
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      st = set_error(LQCD_EHIP, "bandwidth probe launch failed");
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (r > 0 && ms < best) best = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(a);
  (void)hipFree(b);
  if (st != LQCD_OK) return st;
  *gbs = (double)(kind == 1 ? 2 : 1) * (double)(n * 16) / (best * 1e-3) / 1e9;
  return LQCD_OK;
}

extern "C" int lqcd_set_hop_shape(lqcd_ctx* c, int prec, int block, int split, int xcd_map, int nt) {
  if (!c) return set_error(LQCD_EINVAL, "null argument");
  if (prec < 0 || prec > 2) return set_error(LQCD_EINVAL, "bad precision");
  Entry e;
  e.block = block;
  e.split = split;
  e.remap = xcd_map;
  e.nt = nt;
  if (!valid_for(c, prec, e)) return set_error(LQCD_EINVAL, "bad hop launch shape for this lattice");
  c->hop_block[prec] = block;
  c->hop_split[prec] = split;
  c->hop_remap[prec] = xcd_map;
  c->hop_nt[prec] = nt;
  return LQCD_OK;
}

extern "C" int lqcd_get_hop_shape(lqcd_ctx* c, int prec, int* block, int* split, int* xcd_map, int* nt) {
  if (!c) return set_error(LQCD_EINVAL, "null argument");
  if (prec < 0 || prec > 2) return set_error(LQCD_EINVAL, "bad precision");
  if (block) *block = c->hop_block[prec];
  if (split) *split = c->hop_split[prec];
  if (xcd_map) *xcd_map = c->hop_remap[prec];
  if (nt) *nt = c->hop_nt[prec];
  return LQCD_OK;
}
