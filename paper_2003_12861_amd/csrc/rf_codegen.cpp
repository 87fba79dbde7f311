// rf_codegen.cpp -- emits the HIP source of one fused likelihood kernel for a
// lowered graph.
//
// The emitted kernel evaluates the whole node program for each event in
// registers (the paper's batch evaluation of Section 4.1, fused across nodes
// instead of one array pass per node), then -log p and -- for the gradient
// entry point -- a reverse sweep over the same program.
//
// Gradient decomposition.  For a PDF leaf l with normalised value
// v_l = u_l / N_l, d p / d(theta) through l equals
//     (dp/dv_l) v_l [ d log u_l / d(theta) - d log N_l / d(theta) ].
// With w_l = (d log p / d v_l) v_l (the reverse sweep's adjoint times v_l) the
// gradient of NLL = -sum log p is
//     g = -sum_i sum_l w_l,i d log u_l,i / d(theta)  +  sum_l W_l d log N_l / d(theta),
//     W_l = sum_i w_l,i.
// So the event loop only accumulates D_slot = sum_i w_l,i d log u_l,i / d(input)
// per theta-dependent shape input and W_l per leaf (plus the fraction terms of
// sums of PDFs); the FP64 epilogue contracts them with the prologue's
// d log N / d(input) and with d(input)/d(theta).  Normalisation derivatives
// never enter the event loop.
#include <cstdio>
#include <functional>
#include <sstream>

#include "rf_internal.h"

namespace rf {

#include "_gen/rf_device_src.inc"  // RF_DEV_SRC_KABI, _OPS, _MLP, _BODY

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
  }
  return "";
}

static bool blockwide(const Node& n) { return n.op == RF_OP_NUMCONV_BW_CB || n.op == RF_OP_MLP; }

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
  }
}

std::string generate_source(const Lowered& L, int BS, int U) {
  const auto& g = L.nodes;
  const int N = (int)g.size();
  const bool f32 = L.precision == RF_FP32_COMP;
  std::ostringstream o;
  o << "// generated by rfgpu: one fused likelihood kernel\n";
  o << RF_DEV_SRC_KABI << "\n" << RF_DEV_SRC_OPS << "\n";
  if (L.has_mlp) o << RF_DEV_SRC_MLP << "\n#define RF_NSPLIT 3\n";
  o << "#define RF_T " << (f32 ? "float" : "double") << "\n";
  o << "#define RF_NCOL " << L.n_cols << "\n";
  o << "#define RF_NCST " << L.n_cst << "\n";
  o << "#define RF_NSUM " << L.n_sums << "\n";
  o << "#define RF_P " << L.n_params << "\n";
  o << "#define RF_BS " << BS << "\n";
  o << "#define RF_PF " << U << "\n";
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
    any_tab = true;
    o << "__shared__ RF_TABT rf_tab_" << id << "[" << (int)g[id].attrs[2] << " * NumconvRow<RF_TABT>::stride];\n";
  }
  if (any_tab) o << "__shared__ double rf_scr[RF_BS / 64 * 6];\n\n";

  // ---- per-event constants ----
  o << "template <typename T> struct KS {\n";
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    if (is_leaf(g[id].op)) o << "  " << ktype(g[id]) << " l" << id << ";\n";
    if (g[id].op == RF_OP_ADD_PDF) o << "  T a" << id << "[" << (g[id].in.size() + 1) / 2 << "];\n";
  }
  o << "  int unused_;\n";
  o << "  RF_DEV KS load(const double* C) {\n    KS k;\n";
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    if (g[id].op == RF_OP_MLP)
      o << "    k.l" << id << " = MlpK<T>::make(C + " << L.cst_off[id] << ", &rf_mlp_" << id << ", rf_mlpsav_" << id << ");\n";
    else if (blockwide(g[id]))
      o << "    k.l" << id << " = " << ktype(g[id]) << "::make(C + " << L.cst_off[id] << ", rf_tab_" << id << ");\n";
    else if (is_leaf(g[id].op))
      o << "    k.l" << id << " = " << ktype(g[id]) << "::load(C + " << L.cst_off[id] << ");\n";
    if (g[id].op == RF_OP_ADD_PDF) {
      const int nc = ((int)g[id].in.size() + 1) / 2;
      for (int j = 0; j < nc; ++j) o << "    k.a" << id << "[" << j << "] = (T)C[" << L.cst_off[id] + j << "];\n";
    }
  }
  o << "    k.unused_ = 0;\n    return k;\n  }\n};\n\n";

  // ---- prologue ----
  o << "RF_DEV void rf_prologue(const double* th, double* cst, const RfArgs& a) {\n";
  o << "  const int tid = threadIdx.x;\n";
  emit_paramlike(o, L, "  ");
  int item = 0;
  const int NW = BS / 64;
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    const Node& n = g[id];
    if (!is_leaf(n.op) && n.op != RF_OP_ADD_PDF) continue;
    if (blockwide(n)) continue;
    const int tid = 64 * (item % NW) + item / NW;
    ++item;
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
    if (n.op == RF_OP_MLP) {
      o << "    const double box[12] = {";
      for (int j = 0; j < 12; ++j) o << (j ? ", " : "") << dstr(n.attrs[j]);
      o << "};\n    mlp_prologue<RF_BS>(in, box, a.aux + " << L.aux_off[id] + 2 * (int)n.attrs[12]
        << ", (const unsigned short*)a.weights, cst + " << L.cst_off[id] << ", rf_mlp_" << id << ", rf_mlpqs_" << id
        << ");\n  }\n";
      continue;
    }
    o << "    numconv_prologue<RF_BS, RF_TABT>(in, " << dstr(ob.lo) << ", " << dstr(ob.hi) << ", "
      << (int)n.attrs[2] << ", a.aux + " << L.aux_off[id] << ", cst + " << L.cst_off[id] << ", rf_tab_" << id
      << ", rf_scr);\n  }\n";
  }
  o << "  (void)a; (void)tid; (void)cst;\n}\n\n";

  // ---- per-event program ----
  o << "template <typename T, int MODE>\n";
  o << "RF_DEV bool rf_eval(const T* x, const KS<T>& k, double* acc, T* pout, bool valid) {\n";
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    const Node& n = g[id];
    const std::string v = "v" + std::to_string(id);
    if (is_leaf(n.op)) {
      o << "  T d" << id << "[" << leaf_n_shape(n) << "];\n";
      o << "  const T " << v << " = " << eval_call(n, id, "x[" + std::to_string(g[n.in[0]].index) + "]")
        << " * k.l" << id << ".invN;\n";
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
  o << "  const T p = v" << L.top << ";\n";
  o << "  *pout = p;\n";
  o << "  if (!valid) return true;\n";
  o << "  if (!(p > RM<T>::tiny()) || !RM<T>::finite(p)) return false;\n";
  o << "  if (MODE == 0) return true;\n";
  o << "  acc[0] -= (double)RM<T>::log(p);\n";
  o << "  if (MODE == 2) {\n";
  for (int id = 0; id < N; ++id)
    if (L.reach[id] && is_pdf(g[id].op) && id != L.top) o << "    T b" << id << " = (T)0;\n";
  o << "    const T b" << L.top << " = RM<T>::rcp(p);\n";
  // slot lookup
  auto slot_sum = [&](int node, int j) {
    for (const Slot& s : L.slots)
      if (s.node == node && s.j == j) return s.sum;
    return -1;
  };
  for (int id = N - 1; id >= 0; --id) {
    if (!L.reach[id]) continue;
    const Node& n = g[id];
    const std::string b = "b" + std::to_string(id);
    if (n.op == RF_OP_ADD_PDF) {
      const int nc = ((int)n.in.size() + 1) / 2;
      for (int j = 0; j < nc; ++j) o << "    b" << n.in[j] << " += " << b << " * k.a" << id << "[" << j << "];\n";
      for (int j = 0; j < nc - 1; ++j) {
        const int s = slot_sum(id, j);
        if (s >= 0) o << "    acc[" << s << "] += (double)(" << b << " * (v" << n.in[j] << " - v" << n.in[nc - 1] << "));\n";
      }
    } else if (n.op == RF_OP_PROD_PDF) {
      for (size_t j = 0; j < n.in.size(); ++j) {
        o << "    b" << n.in[j] << " += " << b;
        for (size_t i = 0; i < n.in.size(); ++i)
          if (i != j) o << " * v" << n.in[i];
        o << ";\n";
      }
    } else if (is_leaf(n.op) && L.wsum[id] >= 0) {
      o << "    {\n      const T w = " << b << " * v" << id << ";\n";
      for (int j = 0; j < leaf_n_shape(n); ++j) {
        const int s = slot_sum(id, j);
        if (s >= 0) o << "      acc[" << s << "] += (double)(w * d" << id << "[" << j << "]);\n";
      }
      o << "      acc[" << L.wsum[id] << "] += (double)w;\n    }\n";
    }
  }
  o << "  }\n  return true;\n}\n\n";

  // ---- epilogue ----
  o << "template <int MODE>\n";
  o << "RF_DEV void rf_epilogue(const double* S, const double* cst, const double* th, double* out, unsigned nbad) {\n";
  o << "  out[0] = S[0];\n";
  o << "  out[" << L.n_params + 1 << "] = (double)nbad;\n";
  o << "  if (MODE != 2) return;\n";
  emit_paramlike(o, L, "  ");
  o << "  double g[" << (L.n_params > 0 ? L.n_params : 1) << "];\n";
  o << "  for (int k2 = 0; k2 < " << L.n_params << "; ++k2) g[k2] = 0.0;\n";
  for (const Slot& s : L.slots) {
    const Node& n = g[s.node];
    std::string gs;
    if (is_leaf(n.op))
      gs = "-S[" + std::to_string(s.sum) + "] + S[" + std::to_string(L.wsum[s.node]) + "] * cst[" +
           std::to_string(L.cst_off[s.node] + 1 + s.j) + "]";
    else
      gs = "-S[" + std::to_string(s.sum) + "]";
    o << "  {\n    const double gs = " << gs << ";\n";
    emit_jac(o, L, s.pl, "gs");
    o << "  }\n";
  }
  o << "  for (int k2 = 0; k2 < " << L.n_params << "; ++k2) out[1 + k2] = g[k2];\n";
  o << "  for (int j = 0; j < RF_NSUM; ++j) out[" << L.n_params + 2 << " + j] = S[j];\n";
  o << "  (void)cst; (void)th;\n}\n\n";

  o << RF_DEV_SRC_BODY << "\n";
  return o.str();
}

}  // namespace rf
