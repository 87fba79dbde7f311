// rf_jit.cpp -- builds and loads the code object of a generated kernel.
//
// Code objects are content-addressed: the file name is a 64-bit FNV-1a hash
// of the generated source, the compiler flags and the library version.  A hit
// loads the file; a miss runs the ROCm compiler (hipcc --genco for gfx950) in
// a child process and renames its output into place, so concurrent builders
// never see a partial file.  The cache directory is $RFGPU_CACHE_DIR or
// <directory of this library>/_jit.
#include <dlfcn.h>
#include <fcntl.h>
#include <cerrno>
#include <spawn.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "rf_internal.h"

extern char** environ;

namespace rf {

static const char* kFlags[] = {"--genco", "--offload-arch=gfx950", "-O3", "-std=c++17",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-Wno-unused-variable", "-Wno-unused-parameter", "-w"};

uint64_t fnv1a(const std::string& s) {
  uint64_t h = 1469598103934665603ull;
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

static std::string lib_dir() {
  Dl_info info;
  if (dladdr((void*)&fnv1a, &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    size_t k = p.rfind('/');
    if (k != std::string::npos) return p.substr(0, k);
  }
  return ".";
}

std::string cache_dir() {
  const char* e = getenv("RFGPU_CACHE_DIR");
  std::string d = (e && *e) ? std::string(e) : lib_dir() + "/_jit";
  mkdir(d.c_str(), 0755);
  return d;
}

static std::string compiler() {
  const char* e = getenv("RFGPU_HIPCC");
  if (e && *e) return e;
  const char* r = getenv("ROCM_PATH");
  return std::string(r && *r ? r : "/opt/rocm") + "/bin/hipcc";
}

static bool exists(const std::string& p) {
  struct stat st;
  return stat(p.c_str(), &st) == 0 && st.st_size > 0;
}

int build_code_object(const std::string& src, std::string& path) {
  std::string key = src;
  for (const char* f : kFlags) key += std::string(" ") + f;
  key += rf_version();
  char hex[32];
  snprintf(hex, sizeof hex, "%016llx", (unsigned long long)fnv1a(key));
  const std::string dir = cache_dir();
  path = dir + "/" + hex + ".co";
  if (exists(path)) return RF_OK;
  const std::string spath = dir + "/" + hex + ".hip";
  {
    std::ofstream f(spath, std::ios::binary);
    f << src;
    if (!f) return fail(RF_E_DEVICE, "cannot write generated source to " + spath);
  }
  const std::string tmp = path + ".tmp" + std::to_string(getpid());
  const std::string logp = dir + "/" + hex + ".log";
  const std::string cc = compiler();
  std::vector<std::string> args = {cc};
  for (const char* fl : kFlags) args.push_back(fl);
  args.push_back(spath);
  args.push_back("-o");
  args.push_back(tmp);
  std::vector<char*> argv;
  for (auto& a : args) argv.push_back(const_cast<char*>(a.c_str()));
  argv.push_back(nullptr);
  posix_spawn_file_actions_t fa;
  posix_spawn_file_actions_init(&fa);
  posix_spawn_file_actions_addopen(&fa, 1, logp.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
  posix_spawn_file_actions_adddup2(&fa, 1, 2);
  pid_t pid;
  int rc = posix_spawn(&pid, cc.c_str(), &fa, nullptr, argv.data(), environ);
  posix_spawn_file_actions_destroy(&fa);
  if (rc != 0) return fail(RF_E_DEVICE, "cannot start the kernel compiler " + cc);
  int status = 0;
  while (waitpid(pid, &status, 0) < 0 && errno == EINTR) {
  }
  if (!WIFEXITED(status) || WEXITSTATUS(status) != 0 || !exists(tmp)) {
    std::ifstream lf(logp);
    std::stringstream ss;
    ss << lf.rdbuf();
    std::string msg = ss.str();
    if (msg.size() > 2000) msg = msg.substr(0, 2000);
    unlink(tmp.c_str());
    return fail(RF_E_DEVICE, "kernel compilation failed (" + spath + "):\n" + msg);
  }
  if (rename(tmp.c_str(), path.c_str()) != 0) return fail(RF_E_DEVICE, "cannot move code object into the cache");
  return RF_OK;
}

int load_module(const std::string& path, bool f32, Module& m) {
  std::ifstream f(path, std::ios::binary);
  std::vector<char> bytes((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  if (bytes.empty()) return fail(RF_E_DEVICE, "empty code object " + path);
  hipError_t e = hipModuleLoadData(&m.mod, bytes.data());
  if (e != hipSuccess) return hip_fail(e, "hipModuleLoadData");
  const std::string sfx = f32 ? "_f32" : "_f64";
  const std::string kv = "rf_k_values" + sfx, kn = "rf_k_nll" + sfx, kg = "rf_k_grad" + sfx;
  if ((e = hipModuleGetFunction(&m.k_values, m.mod, kv.c_str())) != hipSuccess) return hip_fail(e, kv.c_str());
  if ((e = hipModuleGetFunction(&m.k_nll, m.mod, kn.c_str())) != hipSuccess) return hip_fail(e, kn.c_str());
  if ((e = hipModuleGetFunction(&m.k_grad, m.mod, kg.c_str())) != hipSuccess) return hip_fail(e, kg.c_str());
  return RF_OK;
}

}  // namespace rf
