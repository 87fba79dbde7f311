// rf_graph.cpp -- graph construction, validation and lowering to a flat
// node program (constant-block layout, adjoint sum layout).
//
// The graph follows the paper's description of a RooFit model: observables,
// parameters, functions and PDFs linked into a graph whose every node
// evaluates to a real number (Section 1, Fig. 1).  Lowering splits it the way
// the paper's node caching does (Section 4): parameter-only branches (the
// parameter-like nodes and every normalisation integral) go to the FP64
// prologue; observable-dependent nodes form the per-event program.
#include <cmath>
#include <cstring>
#include <functional>

#include "rf_internal.h"

namespace rf {

static thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? RF_E_OOM : RF_E_DEVICE;
}
const char* last_error() { return g_err.c_str(); }

bool is_leaf(int op) { return op >= RF_OP_GAUSS && op <= RF_OP_POISSON; }
bool is_pdf(int op) { return is_leaf(op) || op == RF_OP_ADD_PDF || op == RF_OP_PROD_PDF; }
bool is_paramlike(int op) {
  return op == K_PARAM || op == K_CONST || op == RF_OP_FN_LINEAR || op == RF_OP_FN_PRODUCT || op == RF_OP_FN_RATIO;
}
int leaf_n_shape(const Node& n) { return (int)n.in.size() - 1; }

// number of FP64 constants of a leaf's block
static int leaf_ncst(const Node& n) {
  switch (n.op) {
    case RF_OP_GAUSS: return 5;
    case RF_OP_CHEB: return 3 + 2 * leaf_n_shape(n);
    case RF_OP_EXP: return 5;
    case RF_OP_DECAY_GAUSS: return 12;
    case RF_OP_ARGUS: return 6;
    case RF_OP_BW: return 6;
    case RF_OP_NUMCONV_BW_CB: return 8;
    case RF_OP_POISSON: return 5;
    case RF_OP_MLP: return 23;  // 8 + the analytic base's constants
  }
  return 0;
}

static int check_leaf(const std::vector<Node>& g, const Node& n) {
  const int ns = leaf_n_shape(n);
  auto want = [&](int nin, int nat) -> int {
    if ((int)n.in.size() != nin) return fail(RF_E_INVALID, "node '" + n.name + "': wrong number of inputs");
    if (nat >= 0 && (int)n.attrs.size() != nat) return fail(RF_E_INVALID, "node '" + n.name + "': wrong number of attributes");
    return RF_OK;
  };
  int rc = RF_OK;
  switch (n.op) {
    case RF_OP_GAUSS: rc = want(3, 0); break;
    case RF_OP_CHEB:
      if (ns < 1 || ns > 8) return fail(RF_E_INVALID, "chebyshev: 1..8 coefficients");
      rc = want(1 + ns, 0);
      break;
    case RF_OP_EXP:
      rc = want(2, 1);
      if (!rc && n.attrs[0] != 0.0 && n.attrs[0] != 1.0) return fail(RF_E_INVALID, "exp: attrs[0] must be 0 (tau) or 1 (rate)");
      break;
    case RF_OP_DECAY_GAUSS: rc = want(4, 0); break;
    case RF_OP_ARGUS:
      rc = want(3, 0);
      if (!rc && g[n.in[1]].op != K_CONST) return fail(RF_E_INVALID, "argus: m0 must be a constant");
      break;
    case RF_OP_BW: rc = want(3, 0); break;
    case RF_OP_NUMCONV_BW_CB:
      rc = want(6, 3);
      if (!rc) {
        const int K = (int)n.attrs[2];
        if (!(n.attrs[0] < n.attrs[1]) || K < 2 || K > 1024 || (double)K != n.attrs[2])
          return fail(RF_E_INVALID, "numconv: attrs (ylo < yhi, integer K in [2, 1024])");
      }
      break;
    case RF_OP_POISSON: {
      rc = want(2, 0);
      const Node& ob = g[n.in[0]];
      if (!rc && !(ob.lo >= 0 && ob.lo == std::floor(ob.lo) && ob.hi == std::floor(ob.hi) && ob.lo < ob.hi &&
                   ob.hi - ob.lo < 2048))
        return fail(RF_E_INVALID, "poisson: the observable's range needs integer ends, 0 <= lo < hi, hi - lo < 2048");
      break;
    }
    case RF_OP_MLP:
      rc = want(6, 13);
      if (!rc) {
        const int K = (int)n.attrs[12];
        if (K < 2 || K > 4096 || (double)K != n.attrs[12]) return fail(RF_E_INVALID, "mlp: K in [2, 4096]");
        for (int j = 0; j < 6; ++j)
          if (!(n.attrs[2 * j] < n.attrs[2 * j + 1])) return fail(RF_E_INVALID, "mlp: input box lo < hi");
      }
      break;
    default: return fail(RF_E_INVALID, "unknown op");
  }
  if (rc) return rc;
  if (g[n.in[0]].op != K_OBS) return fail(RF_E_INVALID, "node '" + n.name + "': input 0 must be an observable");
  for (int j = 1; j < (int)n.in.size(); ++j)
    if (!is_paramlike(g[n.in[j]].op))
      return fail(RF_E_INVALID, "node '" + n.name + "': shape inputs must be parameters, constants or functions of them");
  return RF_OK;
}

namespace {

// The PDF part of a graph as a tree: a PDF node that feeds several sums or
// products is copied once per use, together with the PDF nodes below it, so
// that every path from the top to a leaf has its own nodes (the adjoint's
// path constants are then single products).  Parameters, observables and
// the reachable parameter functions stay shared; the copies of a node
// compute the same expressions on the same inputs.  Inputs keep smaller ids
// than their users.  orig[new id] is the node's id in g.
int expand_shared(const std::vector<Node>& g, const std::vector<char>& reach, int top, int ext, std::vector<Node>& out,
                  std::vector<int>& orig) {
  const int N = (int)g.size();
  std::vector<int> map(N, -1);
  for (int id = 0; id < N; ++id)
    if (!is_pdf(g[id].op) && g[id].op != RF_OP_EXTENDED && (reach[id] || g[id].op == K_PARAM || g[id].op == K_OBS)) {
      map[id] = (int)out.size();
      out.push_back(g[id]);
      orig.push_back(id);
    }
  for (Node& n : out)
    for (int32_t& i : n.in) i = map[i];  // reachable functions take parameter-like inputs only
  std::function<int(int)> copy = [&](int id) -> int {
    Node n = g[id];
    for (int32_t& i : n.in) i = is_pdf(g[i].op) ? copy(i) : map[i];
    out.push_back(n);
    orig.push_back(id);
    return (int)out.size() - 1;
  };
  int t = copy(top);
  if (ext >= 0) {  // the extended wrapper around the PDF
    Node e = g[ext];
    e.in[0] = t;
    e.in[1] = map[e.in[1]];
    out.push_back(e);
    orig.push_back(ext);
    t = (int)out.size() - 1;
  }
  return t;
}

int lower_impl(const std::vector<Node>& g, int top, int precision, Lowered& L, bool expanded);

}  // namespace

int lower(const std::vector<Node>& g, int top, int precision, Lowered& L) { return lower_impl(g, top, precision, L, false); }

namespace {

int lower_impl(const std::vector<Node>& g, int top, int precision, Lowered& L, bool expanded) {
  if (precision != RF_FP64 && precision != RF_FP32_COMP) return fail(RF_E_INVALID, "unknown precision");
  if (top < 0 || top >= (int)g.size()) return fail(RF_E_INVALID, "top id out of range");
  const int top_in = top;
  // the extended-likelihood wrapper: the program's top is the wrapped PDF, and
  // the epilogue adds nu - N log nu
  int ext_nu = -1;
  if (g[top].op == RF_OP_EXTENDED) {
    const Node& e = g[top];
    if (e.in.size() != 2 || !is_pdf(g[e.in[0]].op) || !is_paramlike(g[e.in[1]].op))
      return fail(RF_E_INVALID, "extended: inputs (pdf, nu parameter-like)");
    ext_nu = e.in[1];
    top = e.in[0];
  }
  if (!is_pdf(g[top].op)) return fail(RF_E_INVALID, "top node is not a PDF");
  L = Lowered();
  L.nodes = g;
  L.top = top;
  L.ext_nu = ext_nu;
  L.precision = precision;
  const int N = (int)g.size();
  for (const Node& n : g) {
    if (n.op == K_OBS) L.n_cols++;
    if (n.op == K_PARAM) {
      L.n_params++;
      L.plo.push_back(n.lo);
      L.phi.push_back(n.hi);
    }
  }
  if (L.n_cols > RF_MAX_COLS) return fail(RF_E_INVALID, "too many observables (max 8)");
  if (L.n_params > RF_MAX_PARAMS) return fail(RF_E_INVALID, "too many parameters (max 64)");
  L.reach.assign(N, 0);
  std::function<void(int)> mark = [&](int id) {
    if (L.reach[id]) return;
    L.reach[id] = 1;
    for (int i : g[id].in) mark(i);
  };
  mark(top);
  if (ext_nu >= 0) mark(ext_nu);
  for (int id = 0; id < N; ++id)
    if (L.reach[id] && g[id].op == RF_OP_EXTENDED) return fail(RF_E_INVALID, "extended: only as the compiled top");

  // observable sets (bit masks) of PDFs; parameter dependence of param-likes
  std::vector<uint32_t> obs(N, 0);
  std::vector<char> dep(N, 0);
  for (int id = 0; id < N; ++id) {
    const Node& n = g[id];
    if (!L.reach[id]) continue;
    if (n.op == K_PARAM) dep[id] = 1;
    if (n.op == RF_OP_FN_LINEAR || n.op == RF_OP_FN_PRODUCT || n.op == RF_OP_FN_RATIO) {
      if (n.in.empty()) return fail(RF_E_INVALID, "function without inputs");
      if (n.op == RF_OP_FN_RATIO && n.in.size() != 2) return fail(RF_E_INVALID, "ratio: inputs (a, b)");
      if (n.op == RF_OP_FN_LINEAR && n.attrs.size() != n.in.size() + 1)
        return fail(RF_E_INVALID, "linear function: attrs = (c0, c1..cn)");
      for (int i : n.in) {
        if (!is_paramlike(g[i].op)) return fail(RF_E_INVALID, "function inputs must be parameter-like");
        dep[id] |= dep[i];
      }
    }
    if (is_leaf(n.op)) {
      int rc = check_leaf(g, n);
      if (rc) return rc;
      obs[id] = 1u << g[n.in[0]].index;
      if (n.op == RF_OP_NUMCONV_BW_CB) L.has_numconv = true;
      if (n.op == RF_OP_POISSON) L.has_poisson = true;
      if (n.op == RF_OP_MLP) { L.has_mlp = true; L.mlp_nodes.push_back(id); }
    }
    if (n.op == RF_OP_PROD_PDF) {
      if (n.in.empty()) return fail(RF_E_INVALID, "product without inputs");
      for (int i : n.in) {
        if (!is_pdf(g[i].op)) return fail(RF_E_INVALID, "product inputs must be PDFs");
        if (obs[id] & obs[i]) return fail(RF_E_INVALID, "product factors must depend on disjoint observables");
        obs[id] |= obs[i];
      }
    }
    if (n.op == RF_OP_ADD_PDF) {
      const int ni = (int)n.in.size();
      if (ni < 3 || (ni % 2) == 0) return fail(RF_E_INVALID, "sum: inputs (pdf_1..pdf_n, f_1..f_{n-1}), n >= 2");
      const int nc = (ni + 1) / 2;
      for (int j = 0; j < nc; ++j) {
        if (!is_pdf(g[n.in[j]].op)) return fail(RF_E_INVALID, "sum: first inputs must be PDFs");
        if (j > 0 && obs[n.in[j]] != obs[n.in[0]]) return fail(RF_E_INVALID, "sum: components must share their observables");
        obs[id] = obs[n.in[0]];
      }
      for (int j = nc; j < ni; ++j)
        if (!is_paramlike(g[n.in[j]].op)) return fail(RF_E_INVALID, "sum: fractions must be parameter-like");
    }
  }
  if (L.has_mlp && L.has_numconv) return fail(RF_E_INVALID, "one graph may not mix the convolution and MLP leaves");

  // constant blocks
  L.cst_off.assign(N, -1);
  int off = 0;
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    const Node& n = g[id];
    if (is_leaf(n.op)) { L.cst_off[id] = off; off += leaf_ncst(n); }
    if (n.op == RF_OP_ADD_PDF) { L.cst_off[id] = off; off += ((int)n.in.size() + 1) / 2; }
  }
  L.n_cst = off;

  // auxiliary FP64 inputs: the Gauss-Legendre rule of every convolution leaf
  // (on its window); for an MLP leaf the rule on x's range followed by the
  // normalisation values [Nhat, dNhat/dq1..5] of every workgroup of the
  // normalisation kernel, written before each launch
  L.aux_off.assign(N, -1);
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    if (g[id].op == RF_OP_NUMCONV_BW_CB) {
      const int K = (int)g[id].attrs[2];
      L.aux_off[id] = (int)L.aux.size();
      L.aux.resize(L.aux.size() + 2 * K);
      gauss_legendre(K, g[id].attrs[0], g[id].attrs[1], &L.aux[L.aux_off[id]], &L.aux[L.aux_off[id] + K]);
    } else if (g[id].op == RF_OP_POISSON) {
      // log k! for the observable's integer range
      const Node& ob = g[g[id].in[0]];
      const int lo = (int)ob.lo, K = (int)ob.hi - lo + 1;
      L.aux_off[id] = (int)L.aux.size();
      for (int k = lo; k < lo + K; ++k) L.aux.push_back(std::lgamma((double)k + 1.0));
    } else if (g[id].op == RF_OP_MLP) {
      const int K = (int)g[id].attrs[12];
      const Node& ob = g[g[id].in[0]];
      L.aux_off[id] = (int)L.aux.size();
      L.aux.resize(L.aux.size() + 2 * K + 6 * mlp_renorm_blocks(K), 0.0);
      gauss_legendre(K, ob.lo, ob.hi, &L.aux[L.aux_off[id]], &L.aux[L.aux_off[id] + K]);
    }
  }
  if (L.has_mlp && precision != RF_FP32_COMP)
    return fail(RF_E_INVALID, "the MLP leaf runs in FP32 (BF16 weights): compile with RF_FP32_COMP");

  // PDF tree: a PDF node may feed one sum or product only
  L.parent.assign(N, -1);
  std::vector<int> users(N, 0);
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id] || (g[id].op != RF_OP_ADD_PDF && g[id].op != RF_OP_PROD_PDF)) continue;
    const Node& n = g[id];
    const int np = n.op == RF_OP_ADD_PDF ? ((int)n.in.size() + 1) / 2 : (int)n.in.size();
    for (int j = 0; j < np; ++j) {
      users[n.in[j]]++;
      L.parent[n.in[j]] = id;
    }
  }
  for (int id = 0; id < N; ++id)
    if (L.reach[id] && users[id] > 1) {
      // a shared PDF node: lower the graph expanded into a tree instead
      if (expanded) return fail(RF_E_INVALID, "internal: a shared PDF node after the expansion");
      std::vector<Node> tree;
      std::vector<int> orig;
      const int t = expand_shared(g, L.reach, top, ext_nu >= 0 ? top_in : -1, tree, orig);
      const int rc = lower_impl(tree, t, precision, L, true);
      if (rc) return rc;
      L.orig = orig;
      return RF_OK;
    }
  // canonical nodes (inputs have smaller ids than their users)
  L.canon.assign(N, -1);
  for (int id = N - 1; id >= 0; --id) {
    if (!L.reach[id] || !is_pdf(g[id].op)) continue;
    const int par = L.parent[id];
    L.canon[id] = (par < 0 || g[par].op == RF_OP_ADD_PDF) ? id : L.canon[par];
  }

  // event sums: 0 = sum log p, then D per theta-dependent leaf input, then Y
  std::vector<char> needy(N, 0);
  int s = 1;
  for (int id = 0; id < N; ++id) {
    if (!L.reach[id]) continue;
    const Node& n = g[id];
    if (is_leaf(n.op)) {
      for (int j = 1; j < (int)n.in.size(); ++j)
        if (dep[n.in[j]]) {
          L.slots.push_back({id, j - 1, n.in[j], s++});
          needy[L.canon[id]] = 1;
        }
    }
    if (n.op == RF_OP_ADD_PDF) {
      const int nc = ((int)n.in.size() + 1) / 2;
      for (int j = 0; j < nc - 1; ++j)
        if (dep[n.in[nc + j]]) {
          L.slots.push_back({id, j, n.in[nc + j], -1});
          needy[n.in[j]] = 1;
          needy[n.in[nc - 1]] = 1;
        }
    }
  }
  L.ysum.assign(N, -1);
  for (int id = 0; id < N; ++id)
    if (needy[id]) L.ysum[id] = s++;
  L.n_sums = s;
  return RF_OK;
}

}  // namespace

void eval_paramlike(const Lowered& L, const double* theta, std::vector<double>& pv) {
  const auto& g = L.nodes;
  pv.assign(g.size(), 0.0);
  for (size_t id = 0; id < g.size(); ++id) {
    const Node& n = g[id];
    if (n.op == K_PARAM) pv[id] = theta[n.index];
    else if (n.op == K_CONST) pv[id] = n.value;
    else if (n.op == RF_OP_FN_LINEAR) {
      double v = n.attrs[0];
      for (size_t j = 0; j < n.in.size(); ++j) v += n.attrs[j + 1] * pv[n.in[j]];
      pv[id] = v;
    } else if (n.op == RF_OP_FN_PRODUCT) {
      double v = 1.0;
      for (int i : n.in) v *= pv[i];
      pv[id] = v;
    } else if (n.op == RF_OP_FN_RATIO) {
      pv[id] = pv[n.in[0]] / pv[n.in[1]];
    }
  }
}

int check_theta(const Lowered& L, const double* theta) {
  for (int k = 0; k < L.n_params; ++k) {
    if (!std::isfinite(theta[k])) return fail(RF_E_DOMAIN, "theta[" + std::to_string(k) + "] is not finite");
    if (theta[k] < L.plo[k] || theta[k] > L.phi[k])
      return fail(RF_E_DOMAIN, "theta[" + std::to_string(k) + "] outside its declared bounds");
  }
  std::vector<double> pv;
  eval_paramlike(L, theta, pv);
  const auto& g = L.nodes;
  if (L.ext_nu >= 0 && !(pv[L.ext_nu] > 0 && std::isfinite(pv[L.ext_nu])))
    return fail(RF_E_DOMAIN, "extended: nu must be > 0");
  for (size_t id = 0; id < g.size(); ++id) {
    if (!L.reach[id]) continue;
    const Node& n = g[id];
    auto in = [&](int j) { return pv[n.in[j]]; };
    const double lo = is_leaf(n.op) ? g[n.in[0]].lo : 0.0;
    if (n.op == RF_OP_FN_RATIO && !(in(1) != 0 && std::isfinite(pv[id])))
      return fail(RF_E_DOMAIN, n.name + ": ratio with a zero denominator or a non-finite result");
    switch (n.op) {
      case RF_OP_POISSON:
        if (!(in(1) > 0)) return fail(RF_E_DOMAIN, n.name + ": lambda must be > 0");
        break;
      case RF_OP_GAUSS:
        if (!(in(2) > 0)) return fail(RF_E_DOMAIN, n.name + ": sigma must be > 0");
        break;
      case RF_OP_EXP:
        if (n.attrs[0] == 0.0 && !(in(1) > 0)) return fail(RF_E_DOMAIN, n.name + ": tau must be > 0");
        break;
      case RF_OP_DECAY_GAUSS:
        if (!(in(1) > 0) || !(in(2) > 0)) return fail(RF_E_DOMAIN, n.name + ": tau and sigma must be > 0");
        break;
      case RF_OP_ARGUS:
        if (!(in(2) <= 0)) return fail(RF_E_DOMAIN, n.name + ": c must be <= 0");
        if (!(in(1) > lo)) return fail(RF_E_DOMAIN, n.name + ": m0 must exceed the range's lower edge");
        break;
      case RF_OP_BW:
        if (!(in(2) > 0)) return fail(RF_E_DOMAIN, n.name + ": Gamma must be > 0");
        break;
      case RF_OP_NUMCONV_BW_CB:
        if (!(in(2) > 0) || !(in(3) > 0) || !(in(4) > 0) || !(in(5) >= 1))
          return fail(RF_E_DOMAIN, n.name + ": need Gamma, sigma, alpha > 0 and n >= 1");
        break;
      case RF_OP_MLP:
        for (int j = 1; j < 6; ++j)
          if (in(j) < n.attrs[2 * j] || in(j) > n.attrs[2 * j + 1])
            return fail(RF_E_DOMAIN, n.name + ": surrogate input outside its training box");
        break;
    }
    for (size_t j = 0; j < n.in.size(); ++j)
      if (is_paramlike(g[n.in[j]].op) && !std::isfinite(pv[n.in[j]]))
        return fail(RF_E_DOMAIN, n.name + ": non-finite input");
  }
  return RF_OK;
}

}  // namespace rf

// ============================================================ C API: graph ==
using namespace rf;

extern "C" {

const char* rf_last_error(void) { return rf::last_error(); }

int rf_graph_new(rf_graph** out) {
  if (!out) return fail(RF_E_INVALID, "out is NULL");
  *out = new rf_graph();
  return RF_OK;
}
void rf_graph_free(rf_graph* g) { delete g; }

static int push(rf_graph* g, Node&& n, int32_t* id) {
  if (g->nodes.size() >= 256) return fail(RF_E_INVALID, "too many nodes (max 256)");
  g->nodes.push_back(std::move(n));
  if (id) *id = (int32_t)g->nodes.size() - 1;
  return RF_OK;
}

int rf_graph_observable(rf_graph* g, const char* name, double lo, double hi, int32_t* id) {
  if (!g) return fail(RF_E_INVALID, "graph is NULL");
  if (!(std::isfinite(lo) && std::isfinite(hi) && lo < hi)) return fail(RF_E_INVALID, "observable range must be finite with lo < hi");
  if (g->n_obs >= RF_MAX_COLS) return fail(RF_E_INVALID, "too many observables (max 8)");
  Node n;
  n.op = K_OBS; n.name = name ? name : ""; n.lo = lo; n.hi = hi; n.index = g->n_obs++;
  return push(g, std::move(n), id);
}

int rf_graph_parameter(rf_graph* g, const char* name, double lo, double hi, int32_t* id) {
  if (!g) return fail(RF_E_INVALID, "graph is NULL");
  if (!(lo <= hi) || std::isnan(lo) || std::isnan(hi)) return fail(RF_E_INVALID, "parameter bounds must satisfy lo <= hi");
  if (g->n_params >= RF_MAX_PARAMS) return fail(RF_E_INVALID, "too many parameters (max 64)");
  Node n;
  n.op = K_PARAM; n.name = name ? name : ""; n.lo = lo; n.hi = hi; n.index = g->n_params++;
  return push(g, std::move(n), id);
}

int rf_graph_constant(rf_graph* g, double value, int32_t* id) {
  if (!g) return fail(RF_E_INVALID, "graph is NULL");
  if (!std::isfinite(value)) return fail(RF_E_INVALID, "constant must be finite");
  Node n;
  n.op = K_CONST; n.value = value; n.name = "const";
  return push(g, std::move(n), id);
}

int rf_graph_node(rf_graph* g, int32_t op, const int32_t* inputs, int32_t n_inputs,
                  const double* attrs, int32_t n_attrs, int32_t* id) {
  if (!g) return fail(RF_E_INVALID, "graph is NULL");
  if (!(is_pdf(op) || op == RF_OP_EXTENDED || op == RF_OP_FN_LINEAR || op == RF_OP_FN_PRODUCT ||
        op == RF_OP_FN_RATIO))
    return fail(RF_E_INVALID, "unknown op");
  if (n_inputs < 0 || n_inputs > 64 || n_attrs < 0 || n_attrs > 64) return fail(RF_E_INVALID, "bad input/attribute count");
  if ((n_inputs && !inputs) || (n_attrs && !attrs)) return fail(RF_E_INVALID, "NULL inputs/attrs");
  Node n;
  n.op = op;
  n.name = "node" + std::to_string(g->nodes.size());
  for (int j = 0; j < n_inputs; ++j) {
    if (inputs[j] < 0 || inputs[j] >= (int32_t)g->nodes.size())
      return fail(RF_E_INVALID, "input id does not name an earlier node");
    n.in.push_back(inputs[j]);
  }
  for (int j = 0; j < n_attrs; ++j) {
    if (!std::isfinite(attrs[j])) return fail(RF_E_INVALID, "attributes must be finite");
    n.attrs.push_back(attrs[j]);
  }
  // arity problems are reported here already when they can be decided locally
  if (is_leaf(op)) {
    if (n_inputs < 1 || g->nodes[inputs[0]].op != K_OBS) return fail(RF_E_INVALID, "leaf input 0 must be an observable");
    int rc = check_leaf(g->nodes, n);
    if (rc) return rc;
  }
  return push(g, std::move(n), id);
}

}  // extern "C"
