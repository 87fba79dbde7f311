// rf_codegen.cpp -- emits the HIP source of one fused likelihood kernel for a
// lowered graph.
//
// The emitted kernel evaluates the whole node program for each event in
// registers (the paper's batch evaluation of Section 4.1, fused across nodes
// instead of one array pass per node), then -log p and -- for the gradient
// entry point -- a reverse sweep over the same program.
//
// Gradient decomposition.  In the event loop a PDF node c has the value u_c
// (a leaf: its unnormalised shape; a product: the product of its factors; a
// sum: sum_j a_j s_j u_j with the component scales s_j = 1/N folded into the
// coefficients), and p = s_top u_top.  The adjoint b_c = (dp/du_c)/p factors
// as P_c beta_c: P_c collects the parameter-only factors along the path from
// the top (coefficients a_j s_j), beta_c the per-event ones (1/p, the other
// factors of a product).  With d_j the leaf's event part of d log u/d(input j)
// (or du/d(input j) for leaves in linear form) and f_j its parameter-only
// factor, the gradient of NLL = -sum log p through input j of leaf l is
//     -P_l [ f_j sum_i beta_l u_l d_j  -  Y_l d log N_l / d(input j) ],
// Y_l = sum_i beta_l u_l (one sum shared by the factors of a product), and
// through fraction a_j of a sum n it is -P_n (s_j Y_j - s_last Y_last).  So
// the event loop accumulates only sum log p, one D sum per theta-dependent
// leaf input and the Y sums; every parameter-only factor and every
// normalisation derivative enters once, in the FP64 epilogue.
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <sstream>

#include "rf_internal.h"

namespace rf {

#include "_gen/rf_device_src.inc"  // RF_DEV_SRC_KABI, _OPS, _MLP, _POISSON, _BODY, _HESS, _HBODY

static std::string dstr(double v) {
  char b[40];
  snprintf(b, sizeof b, "%.17g", v);
  std::string s(b);
  if (s.find_first_of(".eEn") == std::string::npos) s += ".0";
  return s;
}

static std::string ktype(const Node& n) {
  switch (n.op) {
    case RF_OP_GAUSS: return "GaussK<T>";
    case RF_OP_CHEB: return "ChebK<T, " + std::to_string(leaf_n_shape(n)) + ">";
    case RF_OP_EXP: return "ExpK<T>";
    case RF_OP_DECAY_GAUSS: return "DecayK<T>";
    case RF_OP_ARGUS: return "ArgusK<T>";
    case RF_OP_BW: return "BwK<T>";
    case RF_OP_NUMCONV_BW_CB: return "NumconvK<T, RF_TABT>";
    case RF_OP_MLP: return "MlpK<T>";
    case RF_OP_POISSON: return "PoissonK<T>";
  }
  return "void";
}

static std::string eval_call(const Node& n, int id, const std::string& x) {
  const std::string k = "k.l" + std::to_string(id), d = "d" + std::to_string(id);
  switch (n.op) {
    case RF_OP_GAUSS: return "gauss_eval<T>(" + x + ", " + k + ", " + d + ")";
    case RF_OP_CHEB: return "cheb_eval<T, " + std::to_string(leaf_n_shape(n)) + ">(" + x + ", " + k + ", " + d + ")";
    case RF_OP_EXP: return "exp_eval<T, " + std::to_string((int)n.attrs[0]) + ">(" + x + ", " + k + ", " + d + ")";
    case RF_OP_DECAY_GAUSS: return "decay_eval<T>(" + x + ", " + k + ", " + d + ")";
    case RF_OP_ARGUS: return "argus_eval<T>(" + x + ", " + k + ", " + d + ")";
    case RF_OP_BW: return "bw_eval<T>(" + x + ", " + k + ", " + d + ")";
    case RF_OP_NUMCONV_BW_CB:
      return "numconv_eval<T, RF_TABT, " + std::to_string((int)n.attrs[2]) + ">(" + x + ", " + k + ", " + d + ")";
    case RF_OP_MLP: return "mlp_leaf_eval<T, RF_NSPLIT, MODE == 2>(" + x + ", " + k + ", " + d + ")";
    case RF_OP_POISSON: return "poisson_eval<T>(" + x + ", " + k + ", " + d + ")";
  }
  return "";
}

// leaves whose derivative outputs are du/d(input) (linear form)
static bool dlin(const Node& n) { return n.op == RF_OP_CHEB; }

// parameter-only factor f_j of a leaf's derivative output j (FP64 expression)
static std::string dscale(const Node& n, int off, int j) {
  auto c = [&](int k) { return "cst[" + std::to_string(off + k) + "]"; };
  switch (n.op) {
    case RF_OP_GAUSS: return "(" + c(4) + (j == 0 ? " * RF_GW_INV)" : " * RF_GW_INV2)");
    case RF_OP_EXP: return n.attrs[0] == 0.0 ? c(4) : "1.0";
    case RF_OP_BW: return j == 0 ? "2.0" : c(5);
    case RF_OP_CHEB: return "0.5";
    case RF_OP_POISSON: return c(4);  // 1/lambda
  }
  return "1.0";
}

static bool blockwide(const Node& n) {
  return n.op == RF_OP_NUMCONV_BW_CB || n.op == RF_OP_MLP || n.op == RF_OP_POISSON;
}

static std::string prologue_call(const Node& n, const Lowered& L, const std::string& in) {
  const auto& g = L.nodes;
  const Node& ob = g[n.in[0]];
  const std::string lo = dstr(ob.lo), hi = dstr(ob.hi);
  const std::string C = "cst + " + std::to_string(L.cst_off[&n - &g[0]]);
  switch (n.op) {
    case RF_OP_GAUSS: return "gauss_prologue(" + in + ", " + lo + ", " + hi + ", " + C + ")";
    case RF_OP_CHEB: return "cheb_prologue<" + std::to_string(leaf_n_shape(n)) + ">(" + in + ", " + lo + ", " + hi + ", " + C + ")";
    case RF_OP_EXP: return "exp_prologue(" + in + ", " + lo + ", " + hi + ", " + std::to_string((int)n.attrs[0]) + ", " + C + ")";
    case RF_OP_DECAY_GAUSS: return "decay_prologue(" + in + ", " + lo + ", " + hi + ", " + C + ")";
    case RF_OP_ARGUS: return "argus_prologue(" + in + ", " + lo + ", " + hi + ", " + C + ")";
    case RF_OP_BW: return "bw_prologue(" + in + ", " + lo + ", " + hi + ", " + C + ")";
  }
  return "";
}

// "const double pvN = ...;" lines for every reachable parameter-like node
static void emit_paramlike(std::ostringstream& o, const Lowered& L, const char* indent) {
  const auto& g = L.nodes;
  for (size_t id = 0; id < g.size(); ++id) {
    if (!L.reach[id]) continue;
    const Node& n = g[id];
    const std::string v = "pv" + std::to_string(id);
    if (n.op == K_PARAM) o << indent << "const double " << v << " = th[" << n.index << "];\n";
    else if (n.op == K_CONST) o << indent << "const double " << v << " = " << dstr(n.value) << ";\n";
    else if (n.op == RF_OP_FN_LINEAR) {
      o << indent << "const double " << v << " = " << dstr(n.attrs[0]);
      for (size_t j = 0; j < n.in.size(); ++j) o << " + " << dstr(n.attrs[j + 1]) << " * pv" << n.in[j];
      o << ";\n";
    } else if (n.op == RF_OP_FN_PRODUCT) {
      o << indent << "const double " << v << " = 1.0";
      for (int i : n.in) o << " * pv" << i;
      o << ";\n";
    } else if (n.op == RF_OP_FN_RATIO) {
      o << indent << "const double " << v << " = pv" << n.in[0] << " / pv" << n.in[1] << ";\n";
    }
  }
}

// g[k] += expr * d(pv_id)/d(theta_k), expanded through the functions
static void emit_jac(std::ostringstream& o, const Lowered& L, int id, const std::string& expr) {
  const Node& n = L.nodes[id];
  if (n.op == K_PARAM) {
    o << "    g[" << n.index << "] += " << expr << ";\n";
  } else if (n.op == RF_OP_FN_LINEAR) {
    for (size_t j = 0; j < n.in.size(); ++j)
      emit_jac(o, L, n.in[j], "(" + expr + ") * " + dstr(n.attrs[j + 1]));
  } else if (n.op == RF_OP_FN_PRODUCT) {
    for (size_t j = 0; j < n.in.size(); ++j) {
      std::string others = "1.0";
      for (size_t i = 0; i < n.in.size(); ++i)
        if (i != j) others += " * pv" + std::to_string(n.in[i]);
      emit_jac(o, L, n.in[j], "(" + expr + ") * " + others);
    }
  } else if (n.op == RF_OP_FN_RATIO) {  // d(a/b) = da / b - (a/b) db / b
    const std::string a = "pv" + std::to_string(n.in[0]), b = "pv" + std::to_string(n.in[1]);
    emit_jac(o, L, n.in[0], "(" + expr + ") / " + b);
    emit_jac(o, L, n.in[1], "-(" + expr + ") * (" + a + " / " + b + ") / " + b);
  }
}

std::vector<int> unfused_slots(const Lowered& L) {
  std::vector<int> slot(L.nodes.size(), -1);
  int ns = 0;
  for (size_t id = 0; id < L.nodes.size(); ++id)
    if (L.reach[id] && is_pdf(L.nodes[id].op)) slot[id] = ns++;
  return slot;
}

// The paper's batch mode (one call per node computes the node's values for all
// events into an array, Section 4.1), as an ablation of the fused kernel:
// kernel rf_u<id> per PDF node in node order (inputs before users) writes
// node id's value of every event to a.values + slot * n; rf_u_nll sums
// log p of the top's array per workgroup into a.part (sums, then bad-event
// counts at a.part + nblk_max), and rf_u_sum adds the partials in a fixed
// order into a.out = [NLL, bad events].  Same per-node arithmetic as rf_eval,
// and the same FP64 re-evaluation of FP32 events below the tail threshold.
static void emit_unfused(std::ostringstream& o, const Lowered& L) {
  const auto& g = L.nodes;
  const int N = (int)g.size();
  const std::vector<int> slot = unfused_slots(L);
  const bool top_add = g[L.top].op == RF_OP_ADD_PDF;
  auto arr = [&](int id) { return "((const RF_T*)a.values + (int64_t)" + std::to_string(slot[id]) + " * a.n)"; };
  const char* head =
      "  typedef RF_T T;\n"
      "  __shared__ double cst[RF_NCST > 0 ? RF_NCST : 1];\n"
      "  rf_prologue(a.theta, cst, a);\n"
      "  __syncthreads();\n"
      "  const KS<T> k = KS<T>::load(cst);\n"
      "  const int64_t step = (int64_t)gridDim.x * RF_BS;\n";
  for (int id = 0; id < N; ++id) {
    if (slot[id] < 0) continue;
    const Node& n = g[id];
    o << "extern \"C\" __global__ __launch_bounds__(RF_BS) void rf_u" << id << "(const RfArgs a) {\n" << head;
    o << "  T* const out = (T*)a.values + (int64_t)" << slot[id] << " * a.n;\n";
    if (is_leaf(n.op)) o << "  const T* const xc = (const T*)a.col[" << g[n.in[0]].index << "];\n";
    o << "  for (int64_t i = (int64_t)blockIdx.x * RF_BS + threadIdx.x; i < a.n; i += step) {\n";
    if (is_leaf(n.op)) {
      o << "    T d" << id << "[" << leaf_n_shape(n) << "];\n";
      o << "    out[i] = " << eval_call(n, id, "xc[i]") << ";\n";
    } else if (n.op == RF_OP_PROD_PDF) {
      o << "    out[i] = ";
      for (size_t j = 0; j < n.in.size(); ++j) o << (j ? " * " : "") << arr(n.in[j]) << "[i]";
      o << ";\n";
    } else {
      const int nc = ((int)n.in.size() + 1) / 2;
      o << "    out[i] = ";
      for (int j = 0; j < nc; ++j) o << (j ? " + " : "") << "k.a" << id << "[" << j << "] * " << arr(n.in[j]) << "[i]";
      o << ";\n";
    }
    o << "  }\n  (void)k;\n}\n\n";
  }
  // NLL kernel: per-workgroup partials of sum w_i log p_i (w_i = 1 without
  // weights), of the bad events and of sum w_i; rows of a.part, nblk_max apart
  o << "extern \"C\" __global__ __launch_bounds__(RF_BS) void rf_u_nll(const RfArgs a) {\n" << head;
  o << "#if RF_TAIL64\n  const KS<double> kd = KS<double>::load(cst);\n#endif\n";
  o << "  const T* const top = " << arr(L.top) << ";\n";
  if (L.weighted) o << "  const T* const wc = (const T*)a.col[" << L.n_cols << "];\n";
  o << "  double s = 0.0, sw = 0.0;\n  unsigned bad = 0;\n";
  o << "  for (int64_t i = (int64_t)blockIdx.x * RF_BS + threadIdx.x; i < a.n; i += step) {\n";
  o << "    const T p = " << (top_add ? "" : "k.stop * ") << "top[i];\n";
  o << "    const double wt = " << (L.weighted ? "(double)wc[i]" : "1.0") << ";\n";
  o << "    if (p > RM<T>::tiny() && p < (T)INFINITY) {\n";
  o << "      s += wt * ((sizeof(T) == 4 ? RF_LN2 : 1.0) * (double)RM<T>::log_acc(p));\n";
  o << "    } else {\n";
  // as in the fused kernel: an FP32 probability below the tail threshold (or
  // not finite) is evaluated again, in FP64, from the event's columns (the
  // weight included, which the per-event program applies itself)
  o << "#if RF_TAIL64\n";
  o << "      double xd[RF_NCOL > 0 ? RF_NCOL : 1], l1 = 0.0, pd;\n";
  o << "      for (int c = 0; c < RF_NCOL; ++c) xd[c] = (double)((const T*)a.col[c])[i];\n";
  o << "      if (rf_eval<double, 1>(xd, kd, &l1, &pd)) s += l1; else ++bad;\n";
  o << "#else\n      ++bad;\n#endif\n";
  o << "    }\n    sw += wt;\n  }\n";
  o << "  __shared__ double ws[RF_BS / 64][3];\n";
  o << "  s = wave_sum(s);\n  sw = wave_sum(sw);\n  const unsigned wb = wave_sum_u(bad);\n";
  o << "  if ((threadIdx.x & 63) == 0) {\n";
  o << "    ws[threadIdx.x >> 6][0] = s; ws[threadIdx.x >> 6][1] = (double)wb; ws[threadIdx.x >> 6][2] = sw;\n  }\n";
  o << "  __syncthreads();\n";
  o << "  if (threadIdx.x == 0) {\n    double t = 0.0, b = 0.0, c = 0.0;\n";
  o << "    for (int w = 0; w < RF_BS / 64; ++w) { t += ws[w][0]; b += ws[w][1]; c += ws[w][2]; }\n";
  o << "    a.part[blockIdx.x] = t;\n    a.part[a.nblk_max + blockIdx.x] = b;\n";
  o << "    a.part[2 * a.nblk_max + blockIdx.x] = c;\n  }\n  (void)k;\n}\n\n";
  o << "// one workgroup: a.out = [NLL, bad events] from the partials, fixed order;\n";
  o << "// an extended program adds nu - N log nu (N: the event count or the sum of\n";
  o << "// the weights)\n";
  o << "extern \"C\" __global__ __launch_bounds__(RF_BS) void rf_u_sum(const RfArgs a, int nb) {\n";
  o << "  __shared__ double ws[RF_BS / 64][3];\n";
  o << "  double s = 0.0, b = 0.0, sw = 0.0;\n";
  o << "  for (int j = threadIdx.x; j < nb; j += RF_BS) {\n";
  o << "    s += a.part[j]; b += a.part[a.nblk_max + j]; sw += a.part[2 * a.nblk_max + j];\n  }\n";
  o << "  s = wave_sum(s);\n  b = wave_sum(b);\n  sw = wave_sum(sw);\n";
  o << "  if ((threadIdx.x & 63) == 0) {\n";
  o << "    ws[threadIdx.x >> 6][0] = s; ws[threadIdx.x >> 6][1] = b; ws[threadIdx.x >> 6][2] = sw;\n  }\n";
  o << "  __syncthreads();\n";
  o << "  if (threadIdx.x == 0) {\n    double t = 0.0, c = 0.0, n_w = 0.0;\n";
  o << "    for (int w = 0; w < RF_BS / 64; ++w) { t += ws[w][0]; c += ws[w][1]; n_w += ws[w][2]; }\n";
  if (L.ext_nu >= 0) {
    o << "    const double* const th = a.theta;\n";
    emit_paramlike(o, L, "    ");
    o << "    const double ext_n = " << (L.weighted ? "n_w" : "th[" + std::to_string(L.n_params) + "]")
      << ", ext_nu = pv" << L.ext_nu << ";\n";
    o << "    a.out[0] = -t + (ext_nu - ext_n * ::log(ext_nu));\n";
  } else {
    o << "    a.out[0] = -t;\n";
  }
  o << "    a.out[1] = c;\n    (void)n_w;\n  }\n}\n";
}

std::string generate_source(const Lowered& L, int BS, int ept, int pfd, int tg, int prio, bool unfused) {
  const auto& g = L.nodes;
  const int N = (int)g.size();
  const bool f32 = L.precision == RF_FP32_COMP;
  std::ostringstream o;
  o << "// generated by rfgpu: one fused likelihood kernel\n";
  o << RF_DEV_SRC_KABI << "\n" << RF_DEV_SRC_OPS << "\n";
  if (L.has_mlp) {
    // BF16 parts per FP32 activation in the surrogate's MFMA products: two
    // keep a 16-bit mantissa (relative 2^-17), far below the network's own
    // error, at two thirds of the MFMA work of three
    int nsplit = 2;
    if (const char* e = getenv("RFGPU_NSPLIT")) {  // tuning override
      const int v = atoi(e);
      if (v == 2 || v == 3) nsplit = v;
    }
    o << RF_DEV_SRC_MLP << "\n#define RF_NSPLIT " << nsplit << "\n";
  }
  if (L.has_poisson) o << RF_DEV_SRC_POISSON << "\n";
  o << "#define RF_T " << (f32 ? "float" : "double") << "\n";
  o << "#define RF_PREC " << (f32 ? "f32" : "f64") << "\n";
  // loaded columns: the observables, then the event weights of a weighted program
  o << "#define RF_NCOL " << L.n_cols + L.weighted << "\n";
  o << "#define RF_NCST " << L.n_cst << "\n";
  o << "#define RF_NSUM " << L.n_sums << "\n";
  o << "#define RF_P " << L.n_params << "\n";
  o << "#define RF_BS " << BS << "\n";
  o << "#define RF_EPT " << ept << "\n";
  o << "#define RF_PFD " << pfd << "\n";
  o << "#define RF_TG " << tg << "\n";
  o << "#define RF_PRIO " << prio << "\n";
  {
    // workgroup reduction through LDS (a table of sums x threads, FP64) in
    // kernels that hold no LDS tables of their own, where it costs no
    // occupancy; there the per-workgroup VALU work it saves matters most
    bool has_tab = L.has_mlp;
    for (int id = 0; id < N; ++id)
      if (L.reach[id] && blockwide(g[id])) has_tab = true;
    int ldsred = ((BS == 256 || BS == 512) && !has_tab && (L.n_sums + 1) * BS * 8 <= 48 * 1024) ? 1 : 0;
    if (const char* e = getenv("RFGPU_LDSRED")) {  // tuning override
      if (atoi(e) == 0) ldsred = 0;
    }
    o << "#define RF_LDSRED " << ldsred << "\n";
  }
  {
    // programs with an MLP leaf: register budget for two wavefronts per SIMD
    // (the LDS allows two; at one, the MFMA and the tanh work of different
    // wavefronts cannot overlap -- measured 1.5x faster with a few spilled
    // values)
    int wpe = L.has_mlp ? 2 : 0;
    if (const char* e = getenv("RFGPU_WPE")) {  // tuning override
      const int v = atoi(e);
      if (v >= 1 && v <= 8) wpe = v;
    }
    o << "#define RF_WPE " << wpe << "\n";
  }
  // programs with an MLP leaf run the event loop in whole wavefronts (the MLP
  // is wave-cooperative) and evaluate in FP32 only (no FP64 re-evaluation)
  o << "#define RF_WAVE_UNIFORM " << (L.has_mlp ? 1 : 0) << "\n";
  o << "#define RF_TAIL64 " << (f32 && !L.has_mlp ? 1 : 0) << "\n";
  o << "#define RF_TABT " << (f32 ? "float" : "double") << "\n\n";
  // LDS tables of block-wide leaves
  bool any_tab = false;
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id] || !blockwide(g[id])) continue;
    if (g[id].op == RF_OP_MLP) {
      o << "__shared__ MlpLds rf_mlp_" << id << ";\n__shared__ float rf_mlpqs_" << id << "[5];\n";
      o << "__shared__ float rf_mlpsav_" << id << "[RF_BS / 64 * 32 * 64];\n";
      continue;
    }
    if (g[id].op == RF_OP_POISSON) {
      const Node& ob = g[g[id].in[0]];
      o << "__shared__ double rf_ptab_" << id << "[" << (int)(ob.hi - ob.lo) + 1 << "];\n";
      o << "__shared__ double rf_pscr_" << id << "[RF_BS / 64 * 2];\n";
      continue;
    }
    any_tab = true;
    o << "__shared__ RF_TABT rf_tab_" << id << "[" << (int)g[id].attrs[2] << " * NumconvRow<RF_TABT>::stride];\n";
  }
  if (any_tab) o << "__shared__ double rf_scr[RF_BS / 64 * 6];\n\n";

  // ---- per-event constants ----
  // scale s_c of a PDF node and path constant P_c, as FP64 expressions over
  // the constant block X
  std::function<std::string(int, const std::string&)> scale = [&](int id, const std::string& X) -> std::string {
    const Node& n = g[id];
    if (is_leaf(n.op)) return X + "[" + std::to_string(L.cst_off[id]) + "]";
    if (n.op == RF_OP_PROD_PDF) {
      std::string r = "1.0";
      for (int i : n.in) r += " * " + scale(i, X);
      return r;
    }
    return "1.0";
  };
  std::function<std::string(int, const std::string&)> pathc = [&](int id, const std::string& X) -> std::string {
    const int par = L.parent[id];
    if (par < 0) return "(" + scale(id, X) + ")";
    const Node& pn = g[par];
    if (pn.op == RF_OP_PROD_PDF) return pathc(par, X);
    const int nc = ((int)pn.in.size() + 1) / 2;
    int j = 0;
    while (j < nc && pn.in[j] != id) ++j;
    return "(" + pathc(par, X) + " * " + X + "[" + std::to_string(L.cst_off[par] + j) + "] * " + scale(id, X) + ")";
  };
  const bool top_add = g[L.top].op == RF_OP_ADD_PDF;
  o << "template <typename T> struct KS {\n";
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    if (is_leaf(g[id].op)) o << "  " << ktype(g[id]) << " l" << id << ";\n";
    if (g[id].op == RF_OP_ADD_PDF) o << "  T a" << id << "[" << (g[id].in.size() + 1) / 2 << "];\n";
  }
  if (!top_add) o << "  T stop;\n";
  o << "  int unused_;\n";
  o << "  RF_DEV KS load(const double* C) {\n    KS k;\n";
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    if (g[id].op == RF_OP_MLP)
      o << "    k.l" << id << " = MlpK<T>::make(C + " << L.cst_off[id] << ", &rf_mlp_" << id << ", rf_mlpsav_" << id << ");\n";
    else if (g[id].op == RF_OP_POISSON)
      o << "    k.l" << id << " = PoissonK<T>::make(C + " << L.cst_off[id] << ", rf_ptab_" << id << ", "
        << (int)g[g[id].in[0]].lo << ", " << (int)(g[g[id].in[0]].hi - g[g[id].in[0]].lo) + 1 << ");\n";
    else if (blockwide(g[id]))
      o << "    k.l" << id << " = " << ktype(g[id]) << "::make(C + " << L.cst_off[id] << ", rf_tab_" << id << ");\n";
    else if (is_leaf(g[id].op))
      o << "    k.l" << id << " = " << ktype(g[id]) << "::load(C + " << L.cst_off[id] << ");\n";
    if (g[id].op == RF_OP_ADD_PDF) {
      // coefficient a_j times the component's scale s_j
      const int nc = ((int)g[id].in.size() + 1) / 2;
      for (int j = 0; j < nc; ++j)
        o << "    k.a" << id << "[" << j << "] = (T)(C[" << L.cst_off[id] + j << "] * " << scale(g[id].in[j], "C") << ");\n";
    }
  }
  if (!top_add) o << "    k.stop = (T)(" << scale(L.top, "C") << ");\n";
  o << "    k.unused_ = 0;\n    return k;\n  }\n};\n\n";

  // ---- prologue ----
  o << "RF_DEV void rf_prologue(const double* th, double* cst, const RfArgs& a) {\n";
  o << "  const int tid = threadIdx.x;\n";
  emit_paramlike(o, L, "  ");
  int item = 0;
  const int NW = BS / 64;
  int n_items = 0;  // prologue items: leaves and sums without block-wide prologues
  for (int id = 0; id < N; ++id)
    if (L.reach[id] && (is_leaf(g[id].op) || g[id].op == RF_OP_ADD_PDF) && !blockwide(g[id])) ++n_items;
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    const Node& n = g[id];
    if (!is_leaf(n.op) && n.op != RF_OP_ADD_PDF) continue;
    if (blockwide(n)) continue;
    const int tid = 64 * (item % NW) + item / NW;
    ++item;
    if (n.op == RF_OP_GAUSS && n_items <= 32 * NW) {
      // two lanes of the wavefront (tid and tid + 32; with at most 32 items
      // per wavefront, lane tid + 32 is no other item's)
      o << "  if (tid == " << tid << " || tid == " << tid + 32 << ") {\n    const double in[] = {";
      for (size_t j = 1; j < n.in.size(); ++j) o << (j > 1 ? ", " : "") << "pv" << n.in[j];
      const Node& ob = g[n.in[0]];
      o << "};\n    gauss_prologue2(in, " << dstr(ob.lo) << ", " << dstr(ob.hi) << ", cst + " << L.cst_off[id]
        << ", tid == " << tid + 32 << ");\n  }\n";
      continue;
    }
    o << "  if (tid == " << tid << ") {\n";
    if (is_leaf(n.op)) {
      o << "    const double in[] = {";
      for (size_t j = 1; j < n.in.size(); ++j) o << (j > 1 ? ", " : "") << "pv" << n.in[j];
      o << "};\n    " << prologue_call(n, L, "in") << ";\n";
    } else {
      const int nc = ((int)n.in.size() + 1) / 2;
      std::string rest = "1.0";
      for (int j = 0; j < nc - 1; ++j) {
        o << "    cst[" << L.cst_off[id] + j << "] = pv" << n.in[nc + j] << ";\n";
        rest += " - pv" + std::to_string(n.in[nc + j]);
      }
      o << "    cst[" << L.cst_off[id] + nc - 1 << "] = " << rest << ";\n";
    }
    o << "  }\n";
  }
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id] || !blockwide(g[id])) continue;
    const Node& n = g[id];
    const Node& ob = g[n.in[0]];
    o << "  {\n    const double in[] = {";
    for (size_t j = 1; j < n.in.size(); ++j) o << (j > 1 ? ", " : "") << "pv" << n.in[j];
    o << "};\n";
    if (n.op == RF_OP_POISSON) {
      o << "    poisson_prologue<RF_BS>(in, " << (int)ob.lo << ", " << (int)(ob.hi - ob.lo) + 1 << ", a.aux + "
        << L.aux_off[id] << ", cst + " << L.cst_off[id] << ", rf_ptab_" << id << ", rf_pscr_" << id << ");\n  }\n";
      continue;
    }
    if (n.op == RF_OP_MLP) {
      o << "    const double box[12] = {";
      for (int j = 0; j < 12; ++j) o << (j ? ", " : "") << dstr(n.attrs[j]);
      o << "};\n    mlp_prologue<RF_BS>(in, box, a.aux + " << L.aux_off[id] + 2 * (int)n.attrs[12] << ", "
        << mlp_renorm_blocks((int)n.attrs[12]) << ", (const unsigned short*)a.weights, cst + " << L.cst_off[id]
        << ", rf_mlp_" << id << ", rf_mlpqs_" << id << ");\n  }\n";
      continue;
    }
    o << "    numconv_prologue<RF_BS, RF_TABT>(in, " << dstr(ob.lo) << ", " << dstr(ob.hi) << ", "
      << (int)n.attrs[2] << ", a.aux + " << L.aux_off[id] << ", cst + " << L.cst_off[id] << ", rf_tab_" << id
      << ", rf_scr);\n  }\n";
  }
  o << "  (void)a; (void)tid; (void)cst;\n}\n\n";

  // ---- per-event program ----
  // returns false when p is not a usable probability (FP32: below 1e-30 or
  // not finite; FP64: not positive or not finite).  With MASK = 1 such an
  // event adds nothing to the sums; with MASK = 0 every event adds its terms
  // unchecked (the caller checks a whole round of events afterwards and
  // discards the round's sums if any event failed).  acc[0] += log p (FP32:
  // log2 p), acc[D], acc[Y].
  o << "template <typename T, int MODE, int MASK = 1>\n";
  o << "RF_DEV bool rf_eval(const T* x, const KS<T>& k, T* acc, T* pout) {\n";
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    const Node& n = g[id];
    const std::string v = "v" + std::to_string(id);
    if (is_leaf(n.op)) {
      o << "  T d" << id << "[" << leaf_n_shape(n) << "];\n";
      o << "  const T " << v << " = " << eval_call(n, id, "x[" + std::to_string(g[n.in[0]].index) + "]") << ";\n";
    } else if (n.op == RF_OP_PROD_PDF) {
      o << "  const T " << v << " = ";
      for (size_t j = 0; j < n.in.size(); ++j) o << (j ? " * " : "") << "v" << n.in[j];
      o << ";\n";
    } else if (n.op == RF_OP_ADD_PDF) {
      const int nc = ((int)n.in.size() + 1) / 2;
      o << "  const T " << v << " = ";
      for (int j = 0; j < nc; ++j) o << (j ? " + " : "") << "k.a" << id << "[" << j << "] * v" << n.in[j];
      o << ";\n";
    }
  }
  o << "  const T p = " << (top_add ? "" : "k.stop * ") << "v" << L.top << ";\n";
  o << "  *pout = p;\n";
  o << "  const bool ok = p > RM<T>::tiny() && p < (T)INFINITY;\n";
  o << "  if (MODE == 0) return ok;\n";
  if (L.weighted) {
    // weighted events: every sum of the event carries its weight, through
    // log p and through r = 1/p, which all adjoint terms share
    o << "  const T wt = x[" << L.n_cols << "];\n";
    o << "  acc[0] += (!MASK || ok) ? wt * RM<T>::log_acc(p) : (T)0;\n";
    // the sum of the weights exists in the gradient mode only (the NLL-only
    // kernel keeps one sum); rf_nll runs the gradient kernel for such programs.
    // A weight enters it only where its event's terms do: an FP32 event
    // below the tail threshold adds its weight in the FP64 re-evaluation
    // instead, so that every weight is counted once (a bad event makes the
    // NLL infinite whatever N is)
    if (L.wsum >= 0) o << "  if (MODE == 2) acc[" << L.wsum << "] += (!MASK || ok) ? wt : (T)0;\n";
    o << "  if (MODE == 2) {\n";
    o << "    const T r = (!MASK || ok) ? RM<T>::rcp(p) * wt : (T)0;\n";
  } else {
    o << "  acc[0] += (!MASK || ok) ? RM<T>::log_acc(p) : (T)0;\n";
    o << "  if (MODE == 2) {\n";
    o << "    const T r = (!MASK || ok) ? RM<T>::rcp(p) : (T)0;\n";
  }
  std::vector<char> declared(N, 0), wdecl(N, 0);
  // beta_c: name of the variable holding it, declared on first use
  std::function<std::string(int)> beta = [&](int id) -> std::string {
    const int par = L.parent[id];
    if (par < 0) return "r";
    if (g[par].op == RF_OP_ADD_PDF) return beta(par);
    const std::string b = "bt" + std::to_string(id);
    if (!declared[id]) {
      const std::string bp = beta(par);
      o << "    const T " << b << " = " << bp;
      for (int i : g[par].in)
        if (i != id) o << " * v" << i;
      o << ";\n";
      declared[id] = 1;
    }
    return b;
  };
  auto wvar = [&](int c) -> std::string {
    const std::string w = "w" + std::to_string(c);
    if (!wdecl[c]) {
      const std::string b = beta(c);
      o << "    const T " << w << " = " << b << " * v" << c << ";\n";
      wdecl[c] = 1;
    }
    return w;
  };
  for (int id = N - 1; id >= 0; --id) {
    if (!L.reach[id] || !is_pdf(g[id].op)) continue;
    if (L.ysum[id] >= 0) {
      const std::string w = wvar(id);
      o << "    acc[" << L.ysum[id] << "] += " << w << ";\n";
    }
    if (!is_leaf(g[id].op)) continue;
    for (const Slot& sl : L.slots) {
      if (sl.node != id || sl.sum < 0) continue;
      const std::string f = dlin(g[id]) ? beta(id) : wvar(L.canon[id]);
      o << "    acc[" << sl.sum << "] += " << f << " * d" << id << "[" << sl.j << "];\n";
    }
  }
  o << "  }\n  return ok;\n}\n\n";

  // ---- epilogue ----
  o << "template <int MODE>\n";
  o << "RF_DEV void rf_epilogue(const double* S, const double* cst, const double* th, double* out, unsigned nbad) {\n";
  if (L.ext_nu >= 0) {
    // extended likelihood: + nu - N log nu, N the number of events (passed
    // after the parameters) or, with weights, their sum over all events
    emit_paramlike(o, L, "  ");
    o << "  const double ext_n = "
      << (L.wsum >= 0 ? "(MODE == 2 ? S[" + std::to_string(L.wsum) + "] : 0.0)"
                      : "th[" + std::to_string(L.n_params) + "]")
      << ", ext_nu = pv" << L.ext_nu << ";\n";
    o << "  out[0] = -S[0] + (ext_nu - ext_n * ::log(ext_nu));\n";
    o << "  out[" << L.n_params + 1 << "] = (double)nbad;\n";
    o << "  if (MODE != 2) return;\n";
  } else {
    o << "  out[0] = -S[0];\n";
    o << "  out[" << L.n_params + 1 << "] = (double)nbad;\n";
    o << "  if (MODE != 2) return;\n";
    emit_paramlike(o, L, "  ");
  }
  o << "  double g[" << (L.n_params > 0 ? L.n_params : 1) << "];\n";
  o << "  for (int k2 = 0; k2 < " << L.n_params << "; ++k2) g[k2] = 0.0;\n";
  for (const Slot& sl : L.slots) {
    const Node& n = g[sl.node];
    std::string gs;
    if (is_leaf(n.op)) {
      const int off = L.cst_off[sl.node];
      gs = "-" + pathc(sl.node, "cst") + " * (" + dscale(n, off, sl.j) + " * S[" + std::to_string(sl.sum) + "] - S[" +
           std::to_string(L.ysum[L.canon[sl.node]]) + "] * cst[" + std::to_string(off + 1 + sl.j) + "])";
    } else {
      const int nc = ((int)n.in.size() + 1) / 2;
      const int cj = n.in[sl.j], cl = n.in[nc - 1];
      gs = "-" + pathc(sl.node, "cst") + " * (" + scale(cj, "cst") + " * S[" + std::to_string(L.ysum[cj]) + "] - " +
           scale(cl, "cst") + " * S[" + std::to_string(L.ysum[cl]) + "])";
    }
    o << "  {\n    const double gs = " << gs << ";\n";
    emit_jac(o, L, sl.pl, "gs");
    o << "  }\n";
  }
  if (L.ext_nu >= 0) {
    o << "  {\n";
    emit_jac(o, L, L.ext_nu, "1.0 - ext_n / ext_nu");
    o << "  }\n";
  }
  o << "  for (int k2 = 0; k2 < " << L.n_params << "; ++k2) out[1 + k2] = g[k2];\n";
  o << "  for (int j = 0; j < RF_NSUM; ++j) out[" << L.n_params + 2 << " + j] = S[j];\n";
  o << "  (void)cst; (void)th;\n}\n\n";

  if (unfused)
    emit_unfused(o, L);
  else
    o << RF_DEV_SRC_BODY << "\n";
  return o.str();
}

// ============================================================ Hessian ==
// The Hessian kernel (its own module, built on first use).  The NLL depends
// on theta only through the slot values a (the theta-dependent leaf inputs
// and fractions), so per event it forms, in FP64 and forward mode over the
// PDF tree, the slot gradient G and slot Hessian H of p (a leaf from its
// second derivatives and those of its normalisation; a product by the
// product rule; a sum linearly, its fractions entering at first order), and
// adds log p, q = G/p and H/p - q q^T to 1 + K + K(K+1)/2 event sums.  The
// epilogue contracts them with the parameter functions' first and second
// derivatives:
//   grad = sum_a g_a J_a,
//   hess = sum_ab H_ab J_a J_b^T + sum_a g_a d2a/dtheta2,
// (g, H the slot gradient and Hessian of the NLL, J_a = da/dtheta), and adds
// the extended term's (N/nu^2) J_nu J_nu^T + (1 - N/nu) d2nu/dtheta2.

bool hess_supported(const Lowered& L, std::string* why) {
  for (size_t id = 0; id < L.nodes.size(); ++id) {
    if (!L.reach[id]) continue;
    const int op = L.nodes[id].op;
    if (op == RF_OP_NUMCONV_BW_CB || op == RF_OP_MLP || op == RF_OP_POISSON) {
      if (why) *why = "no second derivatives for the leaf '" + L.nodes[id].name + "' (convolution, MLP and Poisson leaves)";
      return false;
    }
  }
  if (L.n_params > 16) {
    if (why) *why = "the Hessian takes at most 16 parameters";
    return false;
  }
  return true;
}

int hess_nsums(const Lowered& L) {
  const int K = (int)L.slots.size();
  return 1 + K + K * (K + 1) / 2 + (L.wsum >= 0 ? 1 : 0);
}

// theta-sparse Jacobian of a parameter-like node: (theta index, FP64 factor)
typedef std::vector<std::pair<int, std::string>> SJac;
static SJac sjac(const Lowered& L, int id) {
  const Node& n = L.nodes[id];
  SJac r;
  auto scaled = [&](const SJac& a, const std::string& f) {
    for (const auto& e : a) r.push_back({e.first, "(" + e.second + ") * (" + f + ")"});
  };
  if (n.op == K_PARAM) r.push_back({n.index, "1.0"});
  else if (n.op == RF_OP_FN_LINEAR) {
    for (size_t j = 0; j < n.in.size(); ++j) scaled(sjac(L, n.in[j]), dstr(n.attrs[j + 1]));
  } else if (n.op == RF_OP_FN_PRODUCT) {
    for (size_t j = 0; j < n.in.size(); ++j) {
      std::string o = "1.0";
      for (size_t i = 0; i < n.in.size(); ++i)
        if (i != j) o += " * pv" + std::to_string(n.in[i]);
      scaled(sjac(L, n.in[j]), o);
    }
  } else if (n.op == RF_OP_FN_RATIO) {
    const std::string a = "pv" + std::to_string(n.in[0]), b = "pv" + std::to_string(n.in[1]);
    scaled(sjac(L, n.in[0]), "1.0 / " + b);
    scaled(sjac(L, n.in[1]), "-" + a + " / (" + b + " * " + b + ")");
  }
  return r;
}

// H[k][l] += c * X_k Y_l for sparse X, Y (H row-major at out + P + 2)
static void emit_outer(std::ostringstream& o, const Lowered& L, const SJac& X, const SJac& Y, const std::string& c) {
  const int P = L.n_params;
  for (const auto& x : X)
    for (const auto& y : Y)
      o << "  out[" << P + 2 + x.first * P + y.first << "] += (" << c << ") * (" << x.second << ") * (" << y.second
        << ");\n";
}

// H += c * d2(pv_id)/dtheta2, through the parameter functions
static void emit_hjac(std::ostringstream& o, const Lowered& L, int id, const std::string& c) {
  const Node& n = L.nodes[id];
  if (n.op == RF_OP_FN_LINEAR) {
    for (size_t j = 0; j < n.in.size(); ++j) emit_hjac(o, L, n.in[j], "(" + c + ") * " + dstr(n.attrs[j + 1]));
  } else if (n.op == RF_OP_FN_PRODUCT) {
    const size_t m = n.in.size();
    for (size_t j = 0; j < m; ++j) {
      std::string oj = "1.0";
      for (size_t i = 0; i < m; ++i)
        if (i != j) oj += " * pv" + std::to_string(n.in[i]);
      emit_hjac(o, L, n.in[j], "(" + c + ") * " + oj);
      for (size_t k = 0; k < m; ++k) {
        if (k == j) continue;
        std::string ojk = "1.0";
        for (size_t i = 0; i < m; ++i)
          if (i != j && i != k) ojk += " * pv" + std::to_string(n.in[i]);
        emit_outer(o, L, sjac(L, n.in[j]), sjac(L, n.in[k]), "(" + c + ") * " + ojk);
      }
    }
  } else if (n.op == RF_OP_FN_RATIO) {  // a/b
    const std::string a = "pv" + std::to_string(n.in[0]), b = "pv" + std::to_string(n.in[1]);
    const SJac Ja = sjac(L, n.in[0]), Jb = sjac(L, n.in[1]);
    emit_hjac(o, L, n.in[0], "(" + c + ") / " + b);
    emit_hjac(o, L, n.in[1], "-(" + c + ") * " + a + " / (" + b + " * " + b + ")");
    emit_outer(o, L, Ja, Jb, "-(" + c + ") / (" + b + " * " + b + ")");
    emit_outer(o, L, Jb, Ja, "-(" + c + ") / (" + b + " * " + b + ")");
    emit_outer(o, L, Jb, Jb, "2.0 * (" + c + ") * " + a + " / (" + b + " * " + b + " * " + b + ")");
  }
}

static std::string u2_call(const Node& n, const std::string& x, const std::string& in, const std::string& du,
                           const std::string& d2, const Lowered& L) {
  const Node& ob = L.nodes[n.in[0]];
  const std::string r = ", " + dstr(ob.lo) + ", " + dstr(ob.hi) + ", " + du + ", " + d2 + ")";
  switch (n.op) {
    case RF_OP_GAUSS: return "gauss_u2(" + x + ", " + in + r;
    case RF_OP_CHEB: return "cheb_u2<" + std::to_string(leaf_n_shape(n)) + ">(" + x + ", " + in + r;
    case RF_OP_EXP: return "exp_u2<" + std::to_string((int)n.attrs[0]) + ">(" + x + ", " + in + r;
    case RF_OP_DECAY_GAUSS: return "decay_u2(" + x + ", " + in + r;
    case RF_OP_ARGUS: return "argus_u2(" + x + ", " + in + r;
    case RF_OP_BW: return "bw_u2(" + x + ", " + in + r;
  }
  return "";
}

static std::string n2_call(const Node& n, const std::string& in, const std::string& d2, const Lowered& L) {
  const Node& ob = L.nodes[n.in[0]];
  const std::string r = "(" + in + ", " + dstr(ob.lo) + ", " + dstr(ob.hi) + ", " + d2 + ")";
  switch (n.op) {
    case RF_OP_GAUSS: return "gauss_n2" + r;
    case RF_OP_CHEB: return "cheb_n2<" + std::to_string(leaf_n_shape(n)) + ">" + r;
    case RF_OP_EXP: return "exp_n2<" + std::to_string((int)n.attrs[0]) + ">" + r;
    case RF_OP_DECAY_GAUSS: return "decay_n2" + r;
    case RF_OP_ARGUS: return "argus_n2" + r;
    case RF_OP_BW: return "bw_n2" + r;
  }
  return "";
}

std::string generate_hess_source(const Lowered& L, int BS) {
  const auto& g = L.nodes;
  const int N = (int)g.size();
  const int P = L.n_params;
  const int K = (int)L.slots.size();
  const int NSH = hess_nsums(L);
  const bool f32 = L.precision == RF_FP32_COMP;
  std::ostringstream o;
  o << "// generated by rfgpu: the Hessian kernel of one likelihood program\n";
  o << RF_DEV_SRC_KABI << "\n" << RF_DEV_SRC_OPS << "\n" << RF_DEV_SRC_HESS << "\n";
  o << "#define RF_T " << (f32 ? "float" : "double") << "\n";
  o << "#define RF_NCOL " << L.n_cols + L.weighted << "\n";
  o << "#define RF_NCST " << L.n_cst << "\n";
  o << "#define RF_P " << P << "\n";
  o << "#define RF_BS " << BS << "\n";
  o << "#define RF_NSH " << NSH << "\n";
  // Hessian constants per leaf: its shape input values, then d2N/(N da db)
  std::vector<int> hoff(N, -1);
  int nhc = 0;
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id] || !is_leaf(g[id].op)) continue;
    const int k = leaf_n_shape(g[id]);
    hoff[id] = nhc;
    nhc += k + k * k;
  }
  o << "#define RF_NHC " << nhc << "\n\n";

  // ---- the fused kernels' prologue (N and d log N in cst) ----
  o << "RF_DEV void rf_prologue(const double* th, double* cst, const RfArgs& a) {\n";
  o << "  const int tid = threadIdx.x;\n";
  emit_paramlike(o, L, "  ");
  int item = 0;
  const int NW = BS / 64;
  int n_items = 0;  // prologue items: leaves and sums without block-wide prologues
  for (int id = 0; id < N; ++id)
    if (L.reach[id] && (is_leaf(g[id].op) || g[id].op == RF_OP_ADD_PDF) && !blockwide(g[id])) ++n_items;
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    const Node& n = g[id];
    if (!is_leaf(n.op) && n.op != RF_OP_ADD_PDF) continue;
    const int tid = 64 * (item % NW) + item / NW;
    ++item;
    if (n.op == RF_OP_GAUSS && n_items <= 32 * NW) {
      // two lanes of the wavefront (tid and tid + 32; with at most 32 items
      // per wavefront, lane tid + 32 is no other item's)
      o << "  if (tid == " << tid << " || tid == " << tid + 32 << ") {\n    const double in[] = {";
      for (size_t j = 1; j < n.in.size(); ++j) o << (j > 1 ? ", " : "") << "pv" << n.in[j];
      const Node& ob = g[n.in[0]];
      o << "};\n    gauss_prologue2(in, " << dstr(ob.lo) << ", " << dstr(ob.hi) << ", cst + " << L.cst_off[id]
        << ", tid == " << tid + 32 << ");\n  }\n";
      continue;
    }
    o << "  if (tid == " << tid << ") {\n";
    if (is_leaf(n.op)) {
      o << "    const double in[] = {";
      for (size_t j = 1; j < n.in.size(); ++j) o << (j > 1 ? ", " : "") << "pv" << n.in[j];
      o << "};\n    " << prologue_call(n, L, "in") << ";\n";
    } else {
      const int nc = ((int)n.in.size() + 1) / 2;
      std::string rest = "1.0";
      for (int j = 0; j < nc - 1; ++j) {
        o << "    cst[" << L.cst_off[id] + j << "] = pv" << n.in[nc + j] << ";\n";
        rest += " - pv" + std::to_string(n.in[nc + j]);
      }
      o << "    cst[" << L.cst_off[id] + nc - 1 << "] = " << rest << ";\n";
    }
    o << "  }\n";
  }
  o << "  (void)a; (void)tid; (void)cst;\n}\n\n";

  // ---- Hessian prologue: leaf inputs and d2N/N ----
  o << "RF_DEV void rf_prologue_h(const double* th, const double* cst, double* hc) {\n";
  o << "  const int tid = threadIdx.x;\n";
  emit_paramlike(o, L, "  ");
  item = 0;
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id] || !is_leaf(g[id].op)) continue;
    const Node& n = g[id];
    const int k = leaf_n_shape(n);
    const int tid = 64 * (item % NW) + item / NW;
    ++item;
    o << "  if (tid == " << tid << ") {\n    const double in[] = {";
    for (size_t j = 1; j < n.in.size(); ++j) o << (j > 1 ? ", " : "") << "pv" << n.in[j];
    o << "};\n    double d2[" << k * k << "];\n    " << n2_call(n, "in", "d2", L) << ";\n";
    o << "    for (int j = 0; j < " << k << "; ++j) hc[" << hoff[id] << " + j] = in[j];\n";
    o << "    for (int j = 0; j < " << k * k << "; ++j) hc[" << hoff[id] + k << " + j] = d2[j] * cst["
      << L.cst_off[id] << "];\n  }\n";
  }
  o << "  (void)tid; (void)th; (void)cst; (void)hc;\n}\n\n";

  // ---- per event: value, slot gradient and slot Hessian of every PDF node ----
  // gv[c][a]: name of dv_c/da (absent: zero); hv[c][{a,b}] (a <= b) likewise
  std::vector<std::map<int, std::string>> gv(N);
  std::vector<std::map<std::pair<int, int>, std::string>> hv(N);
  auto pr = [](int a, int b) { return a <= b ? std::make_pair(a, b) : std::make_pair(b, a); };
  int tmp = 0;
  o << "RF_DEV bool rf_eval_h(const double* x, const double* cst, const double* hc, double* acc) {\n";
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id] || !is_pdf(g[id].op)) continue;
    const Node& n = g[id];
    const std::string v = "v" + std::to_string(id);
    if (is_leaf(n.op)) {
      const int k = leaf_n_shape(n), off = L.cst_off[id], ho = hoff[id];
      const std::string u = "u" + std::to_string(id), du = "du" + std::to_string(id), d2 = "dd" + std::to_string(id);
      o << "  double " << du << "[" << k << "], " << d2 << "[" << k * k << "];\n";
      o << "  const double " << u << " = " << u2_call(n, "x[" + std::to_string(g[n.in[0]].index) + "]",
                                                       "hc + " + std::to_string(ho), du, d2, L) << ";\n";
      o << "  const double " << v << " = " << u << " * cst[" << off << "];\n";
      std::vector<std::pair<int, int>> sl;  // (slot, input position)
      for (int a = 0; a < K; ++a)
        if (L.slots[a].node == id) sl.push_back({a, L.slots[a].j});
      auto nj = [&](int j) { return "cst[" + std::to_string(off + 1 + j) + "]"; };
      for (const auto& s : sl) {
        const std::string gn = "g" + std::to_string(id) + "_" + std::to_string(s.first);
        o << "  const double " << gn << " = (" << du << "[" << s.second << "] - " << u << " * " << nj(s.second)
          << ") * cst[" << off << "];\n";
        gv[id][s.first] = gn;
      }
      for (size_t p1 = 0; p1 < sl.size(); ++p1)
        for (size_t p2 = p1; p2 < sl.size(); ++p2) {
          const int j = sl[p1].second, l = sl[p2].second;
          const std::string hn = "h" + std::to_string(id) + "_" + std::to_string(sl[p1].first) + "_" + std::to_string(sl[p2].first);
          o << "  const double " << hn << " = (" << d2 << "[" << j * k + l << "] - " << du << "[" << j << "] * " << nj(l)
            << " - " << du << "[" << l << "] * " << nj(j) << " - " << u << " * hc[" << ho + k + j * k + l << "] + 2.0 * "
            << u << " * " << nj(j) << " * " << nj(l) << ") * cst[" << off << "];\n";
          hv[id][pr(sl[p1].first, sl[p2].first)] = hn;
        }
    } else if (n.op == RF_OP_PROD_PDF) {
      // fold the factors: (f g)'' = f'' g + f' g'^T + g' f'^T + f g''
      std::string cv = "v" + std::to_string(n.in[0]);
      std::map<int, std::string> cg = gv[n.in[0]];
      std::map<std::pair<int, int>, std::string> ch = hv[n.in[0]];
      for (size_t f = 1; f < n.in.size(); ++f) {
        const int F = n.in[f];
        const std::string fv = "v" + std::to_string(F);
        const std::string nv = (f + 1 == n.in.size()) ? v : "t" + std::to_string(tmp++);
        std::map<int, std::string> ng;
        std::map<std::pair<int, int>, std::string> nh;
        for (const auto& e : cg) {
          const std::string t = "t" + std::to_string(tmp++);
          o << "  const double " << t << " = " << e.second << " * " << fv << ";\n";
          ng[e.first] = t;
        }
        for (const auto& e : gv[F]) {
          const std::string t = "t" + std::to_string(tmp++);
          o << "  const double " << t << " = " << cv << " * " << e.second << ";\n";
          ng[e.first] = t;
        }
        for (const auto& e : ch) {
          const std::string t = "t" + std::to_string(tmp++);
          o << "  const double " << t << " = " << e.second << " * " << fv << ";\n";
          nh[e.first] = t;
        }
        for (const auto& e : hv[F]) {
          const std::string t = "t" + std::to_string(tmp++);
          o << "  const double " << t << " = " << cv << " * " << e.second << ";\n";
          nh[e.first] = t;
        }
        for (const auto& a : cg)
          for (const auto& b : gv[F]) {
            const std::string t = "t" + std::to_string(tmp++);
            o << "  const double " << t << " = " << a.second << " * " << b.second << ";\n";
            nh[pr(a.first, b.first)] = t;
          }
        o << "  const double " << nv << " = " << cv << " * " << fv << ";\n";
        cv = nv;
        cg = ng;
        ch = nh;
      }
      gv[id] = cg;
      hv[id] = ch;
    } else {  // ADD
      const int nc = ((int)n.in.size() + 1) / 2, off = L.cst_off[id];
      auto cj = [&](int j) { return "cst[" + std::to_string(off + j) + "]"; };
      o << "  const double " << v << " = ";
      for (int j = 0; j < nc; ++j) o << (j ? " + " : "") << cj(j) << " * v" << n.in[j];
      o << ";\n";
      for (int j = 0; j < nc; ++j) {
        for (const auto& e : gv[n.in[j]]) {
          const std::string t = "t" + std::to_string(tmp++);
          o << "  const double " << t << " = " << cj(j) << " * " << e.second << ";\n";
          gv[id][e.first] = t;
        }
        for (const auto& e : hv[n.in[j]]) {
          const std::string t = "t" + std::to_string(tmp++);
          o << "  const double " << t << " = " << cj(j) << " * " << e.second << ";\n";
          hv[id][e.first] = t;
        }
      }
      const int last = n.in[nc - 1];
      for (int a = 0; a < K; ++a) {
        if (L.slots[a].node != id) continue;
        const int fj = L.slots[a].j, child = n.in[fj];
        const std::string t = "t" + std::to_string(tmp++);
        o << "  const double " << t << " = v" << child << " - v" << last << ";\n";
        gv[id][a] = t;
        // d2 v / d f_j d b = dv_child/db - dv_last/db
        for (const auto& e : gv[child]) hv[id][pr(a, e.first)] = e.second;
        for (const auto& e : gv[last]) {
          const std::string t2 = "t" + std::to_string(tmp++);
          o << "  const double " << t2 << " = -" << e.second << ";\n";
          hv[id][pr(a, e.first)] = t2;
        }
      }
    }
  }
  const int top = L.top;
  o << "  const double p = v" << top << ";\n";
  o << "  if (!(p > 0.0) || !(p < INFINITY)) return false;\n";
  o << "  const double r = 1.0 / p;\n";
  o << "  const double w = " << (L.weighted ? "x[" + std::to_string(L.n_cols) + "]" : std::string("1.0")) << ";\n";
  o << "  acc[0] += w * ::log(p);\n";
  for (int a = 0; a < K; ++a) {
    auto it = gv[top].find(a);
    o << "  const double q" << a << " = " << (it == gv[top].end() ? std::string("0.0") : it->second + " * r") << ";\n";
    o << "  acc[" << 1 + a << "] += w * q" << a << ";\n";
  }
  int idx = 1 + K;
  for (int a = 0; a < K; ++a)
    for (int b = a; b < K; ++b, ++idx) {
      auto it = hv[top].find({a, b});
      o << "  acc[" << idx << "] += w * (" << (it == hv[top].end() ? std::string("0.0") : it->second + " * r") << " - q" << a
        << " * q" << b << ");\n";
    }
  if (L.wsum >= 0) o << "  acc[" << idx << "] += w;\n";
  o << "  return true;\n}\n\n";

  // ---- epilogue: theta-space NLL, gradient and Hessian ----
  o << "RF_DEV void rf_epilogue_h(const double* S, const double* th, double* out, unsigned nbad) {\n";
  emit_paramlike(o, L, "  ");
  if (L.ext_nu >= 0)
    o << "  const double ext_n = " << (L.wsum >= 0 ? "S[" + std::to_string(idx) + "]" : "th[" + std::to_string(P) + "]")
      << ", ext_nu = pv" << L.ext_nu << ";\n";
  o << "  out[0] = -S[0]" << (L.ext_nu >= 0 ? " + (ext_nu - ext_n * ::log(ext_nu))" : "") << ";\n";
  o << "  out[" << P + 1 << "] = (double)nbad;\n";
  std::vector<SJac> J(K);
  for (int a = 0; a < K; ++a) J[a] = sjac(L, L.slots[a].pl);
  for (int a = 0; a < K; ++a) {
    o << "  const double ga" << a << " = -S[" << 1 + a << "];\n";
    for (const auto& e : J[a]) o << "  out[" << 1 + e.first << "] += ga" << a << " * (" << e.second << ");\n";
  }
  idx = 1 + K;
  for (int a = 0; a < K; ++a)
    for (int b = a; b < K; ++b, ++idx) {
      o << "  {\n  const double hab = -S[" << idx << "];\n";
      emit_outer(o, L, J[a], J[b], "hab");
      if (a != b) emit_outer(o, L, J[b], J[a], "hab");
      o << "  }\n";
    }
  for (int a = 0; a < K; ++a) emit_hjac(o, L, L.slots[a].pl, "ga" + std::to_string(a));
  if (L.ext_nu >= 0) {
    const SJac Jn = sjac(L, L.ext_nu);
    for (const auto& e : Jn) o << "  out[" << 1 + e.first << "] += (1.0 - ext_n / ext_nu) * (" << e.second << ");\n";
    emit_outer(o, L, Jn, Jn, "ext_n / (ext_nu * ext_nu)");
    emit_hjac(o, L, L.ext_nu, "1.0 - ext_n / ext_nu");
  }
  o << "  (void)th;\n}\n\n";
  o << RF_DEV_SRC_HBODY << "\n";
  return o.str();
}

}  // namespace rf
