// rf_pycall.cpp -- CPython entry for the synchronous evaluation calls of the
// Python binding (argument marshalling only, like the ctypes binding beside
// it, with less per-call overhead: no ctypes argument conversion, theta read
// in place when it is a float64 vector, the result tuple built here).
//
// The library's functions are not linked: the binding passes the addresses
// that ctypes resolved in the loaded librfgpu.so (init), so both paths call
// the same library instance.  A call whose theta is not n_params numbers
// returns None, and the binding then takes its checked ctypes path, which
// raises the usual errors.
#define PY_SSIZE_T_CLEAN
#include <Python.h>
#define NPY_NO_DEPRECATED_API NPY_1_7_API_VERSION
#include <numpy/arrayobject.h>

#include <cstdint>
#include <initializer_list>

namespace {

typedef int (*NllGradFn)(void* p, const double* theta, double* nll, double* grad, int64_t* n_bad, void* stream);
typedef int (*BinnedNllGradFn)(void* b, const double* theta, double* nll, double* grad, void* stream);

NllGradFn g_nll_grad = nullptr;      // rf_nll_grad
BinnedNllGradFn g_binned_nll_grad = nullptr;
NllGradFn g_sum_nll_grad = nullptr;  // rf_sum_nll_grad (same signature as rf_nll_grad)

constexpr Py_ssize_t kMaxTheta = 256;

// theta as a pointer to n doubles: the array's own data when it is a
// contiguous, aligned float64 vector of n values, else a copy of the
// sequence's values into buf.  Returns nullptr (no Python error set) when
// theta is neither.
const double* theta_ptr(PyObject* o, Py_ssize_t n, double* buf) {
  if (n < 0 || n > kMaxTheta) return nullptr;
  if (PyArray_Check(o)) {
    PyArrayObject* a = (PyArrayObject*)o;
    if (PyArray_TYPE(a) == NPY_DOUBLE && PyArray_NDIM(a) == 1 && PyArray_DIM(a, 0) == n &&
        PyArray_IS_C_CONTIGUOUS(a) && PyArray_ISALIGNED(a))
      return (const double*)PyArray_DATA(a);
  }
  PyObject* seq = PySequence_Fast(o, "theta");
  if (!seq) {
    PyErr_Clear();
    return nullptr;
  }
  const double* r = buf;
  if (PySequence_Fast_GET_SIZE(seq) != n) {
    r = nullptr;
  } else {
    PyObject** items = PySequence_Fast_ITEMS(seq);
    for (Py_ssize_t i = 0; i < n; ++i) {
      buf[i] = PyFloat_AsDouble(items[i]);
      if (buf[i] == -1.0 && PyErr_Occurred()) {
        PyErr_Clear();
        r = nullptr;
        break;
      }
    }
  }
  Py_DECREF(seq);
  return r;
}

bool get_ptr(PyObject* o, void** out) {
  *out = PyLong_AsVoidPtr(o);
  return !(*out == nullptr && PyErr_Occurred());
}

// init(rf_nll_grad, rf_binned_nll_grad, rf_sum_nll_grad): their addresses
PyObject* py_init(PyObject*, PyObject* const* args, Py_ssize_t nargs) {
  if (nargs != 3) {
    PyErr_SetString(PyExc_TypeError, "init(rf_nll_grad, rf_binned_nll_grad, rf_sum_nll_grad)");
    return nullptr;
  }
  void *a, *b, *c;
  if (!get_ptr(args[0], &a) || !get_ptr(args[1], &b) || !get_ptr(args[2], &c)) return nullptr;
  g_nll_grad = (NllGradFn)a;
  g_binned_nll_grad = (BinnedNllGradFn)b;
  g_sum_nll_grad = (NllGradFn)c;
  Py_RETURN_NONE;
}

// the arguments of one call: (handle, theta, n_params, stream) unpacked, and
// the gradient array the call fills
struct Call {
  void* h = nullptr;
  void* stream = nullptr;
  const double* th = nullptr;
  PyArrayObject* g = nullptr;
  double buf[kMaxTheta];
};

// 1: ready; 0: take the checked path (return None); -1: Python error
int unpack(PyObject* const* args, Py_ssize_t nargs, const char* usage, Call& c) {
  if (nargs != 4) {
    PyErr_SetString(PyExc_TypeError, usage);
    return -1;
  }
  if (args[0] == Py_None) return 0;  // a freed handle: the checked path reports it
  if (!get_ptr(args[0], &c.h) || !get_ptr(args[3], &c.stream)) return -1;
  const Py_ssize_t n = PyLong_AsSsize_t(args[2]);
  if (n == -1 && PyErr_Occurred()) return -1;
  if (!c.h) return 0;
  c.th = theta_ptr(args[1], n, c.buf);
  if (!c.th) return 0;
  npy_intp dim = n;
  c.g = (PyArrayObject*)PyArray_SimpleNew(1, &dim, NPY_DOUBLE);
  return c.g ? 1 : -1;
}

// a tuple of the new references in items (all released if one is missing)
PyObject* result(std::initializer_list<PyObject*> items) {
  bool ok = true;
  for (PyObject* o : items) ok = ok && o;
  PyObject* t = ok ? PyTuple_New((Py_ssize_t)items.size()) : nullptr;
  if (!t) {
    for (PyObject* o : items) Py_XDECREF(o);
    return nullptr;
  }
  Py_ssize_t i = 0;
  for (PyObject* o : items) PyTuple_SET_ITEM(t, i++, o);
  return t;
}

// (handle, theta, n_params, stream) -> (rc, nll, grad, n_bad) or None, for
// the entry points with rf_nll_grad's signature
PyObject* call_nll_grad(NllGradFn fn, PyObject* const* args, Py_ssize_t nargs, const char* usage) {
  if (!fn) {
    PyErr_SetString(PyExc_RuntimeError, "rf_pycall.init was not called");
    return nullptr;
  }
  Call c;
  const int u = unpack(args, nargs, usage, c);
  if (u <= 0) {
    if (u < 0) return nullptr;
    Py_RETURN_NONE;
  }
  double nll = 0.0;
  int64_t nb = 0;
  int rc;
  Py_BEGIN_ALLOW_THREADS
  rc = fn(c.h, c.th, &nll, (double*)PyArray_DATA(c.g), &nb, c.stream);
  Py_END_ALLOW_THREADS
  return result({PyLong_FromLong(rc), PyFloat_FromDouble(nll), (PyObject*)c.g, PyLong_FromLongLong(nb)});
}

PyObject* py_nll_grad(PyObject*, PyObject* const* args, Py_ssize_t nargs) {
  return call_nll_grad(g_nll_grad, args, nargs, "nll_grad(handle, theta, n_params, stream)");
}

PyObject* py_sum_nll_grad(PyObject*, PyObject* const* args, Py_ssize_t nargs) {
  return call_nll_grad(g_sum_nll_grad, args, nargs, "sum_nll_grad(handle, theta, n_params, stream)");
}

// binned_nll_grad(handle, theta, n_params, stream) -> (rc, nll, grad) or None
PyObject* py_binned_nll_grad(PyObject*, PyObject* const* args, Py_ssize_t nargs) {
  if (!g_binned_nll_grad) {
    PyErr_SetString(PyExc_RuntimeError, "rf_pycall.init was not called");
    return nullptr;
  }
  Call c;
  const int u = unpack(args, nargs, "binned_nll_grad(handle, theta, n_params, stream)", c);
  if (u <= 0) {
    if (u < 0) return nullptr;
    Py_RETURN_NONE;
  }
  double nll = 0.0;
  int rc;
  Py_BEGIN_ALLOW_THREADS
  rc = g_binned_nll_grad(c.h, c.th, &nll, (double*)PyArray_DATA(c.g), c.stream);
  Py_END_ALLOW_THREADS
  return result({PyLong_FromLong(rc), PyFloat_FromDouble(nll), (PyObject*)c.g});
}

PyMethodDef kMethods[] = {
    {"init", (PyCFunction)(void (*)(void))py_init, METH_FASTCALL, "init(rf_nll_grad, rf_binned_nll_grad, rf_sum_nll_grad)"},
    {"nll_grad", (PyCFunction)(void (*)(void))py_nll_grad, METH_FASTCALL,
     "nll_grad(handle, theta, n_params, stream) -> (rc, nll, grad, n_bad), or None for the checked path"},
    {"sum_nll_grad", (PyCFunction)(void (*)(void))py_sum_nll_grad, METH_FASTCALL,
     "sum_nll_grad(handle, theta, n_params, stream) -> (rc, nll, grad, n_bad), or None for the checked path"},
    {"binned_nll_grad", (PyCFunction)(void (*)(void))py_binned_nll_grad, METH_FASTCALL,
     "binned_nll_grad(handle, theta, n_params, stream) -> (rc, nll, grad), or None for the checked path"},
    {nullptr, nullptr, 0, nullptr}};

PyModuleDef kModule = {PyModuleDef_HEAD_INIT, "_rfcall", "Synchronous evaluation calls of librfgpu (marshalling only).",
                       -1, kMethods};

}  // namespace

PyMODINIT_FUNC PyInit__rfcall(void) {
  import_array();
  return PyModule_Create(&kModule);
}
