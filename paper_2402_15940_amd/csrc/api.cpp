// C ABI of the pafem library: object lifetimes, argument checking, dispatch.
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>

#include "internal.h"

namespace pafem {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

namespace {

inline hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

#define CHECK_ARG(cond, msg)             \
  do {                                   \
    if (!(cond)) {                       \
      set_error(msg);                    \
      return PAFEM_ERR_INVALID_ARG;      \
    }                                    \
  } while (0)

// The element kernels' 1D tables for every order, into constant memory of
// the current device (each kernel source file holds its own copy).
hipError_t upload_basis_tables() {
  std::vector<double> t64(tab_words());
  for (int p = 1; p <= kMaxP; ++p) {
    const int n = p + 1, q = p + 2;
    const int nh = n / 2, nhe = n - nh, qh = q / 2, qhe = q - qh;
    std::vector<double> nodes(n), pts(q), wts(q);
    gll_nodes(p, nodes.data());
    gauss_legendre(q, pts.data(), wts.data());
    double* B = t64.data() + tab_off(p);
    lagrange_tables(n, nodes.data(), q, pts.data(), B, B + q * n);
    // mirror-split tables of B (t = 0) and G (t = 1): sums and differences of
    // mirrored entries, halved; the middle node / point enters once
    for (int t = 0; t < 2; ++t) {
      const double* T = B + t * q * n;
      double* Pf = B + 2 * q * n + t * mir_words(p);
      double* Mf = Pf + qhe * nhe;
      double* Pt = Mf + qhe * nh;
      double* Mt = Pt + nhe * qhe;
      for (int j = 0; j < qhe; ++j)
        for (int i = 0; i < nhe; ++i) {
          const double a = T[j * n + i], b = T[j * n + (n - 1 - i)];
          Pf[j * nhe + i] = i < nh ? 0.5 * (a + b) : a;
          if (i < nh) Mf[j * nh + i] = 0.5 * (a - b);
        }
      for (int i = 0; i < nhe; ++i)
        for (int k = 0; k < qhe; ++k) {
          const double a = T[k * n + i], b = T[(q - 1 - k) * n + i];
          Pt[i * qhe + k] = k < qh ? 0.5 * (a + b) : a;
          if (k < qh) Mt[i * qh + k] = 0.5 * (a - b);
        }
    }
  }
  std::vector<float> t32(t64.begin(), t64.end());
  hipError_t e = upload_tables_apply(t64.data(), t32.data(), t64.size());
  if (e == hipSuccess) e = upload_tables_batched(t64.data(), t32.data(), t64.size());
  if (e == hipSuccess) e = upload_tables_persistent(t64.data(), t32.data(), t64.size());
  return e;
}

int need_device(const Ctx* c) {
  if (c->host_only) {
    set_error("operation needs a GPU context (created with device >= 0)");
    return PAFEM_ERR_UNSUPPORTED;
  }
  PAFEM_TRY_HIP(hipSetDevice(c->device));
  return PAFEM_OK;
}

template <typename T>
int upload(DevBuf& b, const T* src, size_t n) {
  PAFEM_TRY(b.ensure(n * sizeof(T)));
  if (n) PAFEM_TRY_HIP(hipMemcpy(b.ptr, src, n * sizeof(T), hipMemcpyHostToDevice));
  return PAFEM_OK;
}

GeomArgs geom(const Op* op, const double* pts, const double* wts) {
  const Mesh* m = op->space->mesh;
  GeomArgs g;
  g.verts = m->d_verts.as<double>();
  g.nx = m->nx;
  g.ny = m->ny;
  g.nz = m->nz;
  g.ne = op->space->ne;
  g.q = op->q;
  g.pts = pts;
  g.wts = wts;
  return g;
}

// Device table layout (T = double or float): B[q][n] | G[q][n] | pts[q] | wts[q]
template <typename T>
const T* tabB(const DevBuf& b) { return b.as<T>(); }
template <typename T>
const T* tabG(const DevBuf& b, int q, int n) { return b.as<T>() + q * n; }
inline const double* tabPts(const DevBuf& b, int q, int n) { return b.as<double>() + 2 * q * n; }
inline const double* tabWts(const DevBuf& b, int q, int n) {
  return b.as<double>() + 2 * q * n + q;
}

}  // namespace

int ensure_host_maps(Space* sp) {
  if (sp->have_maps) return PAFEM_OK;
  const Mesh* m = sp->mesh;
  try {
    build_restriction(m->nx, m->ny, m->nz, sp->p, sp->E);
    build_restriction_transpose(sp->E, sp->ndofs, sp->et_off, sp->et_idx);
    std::vector<int32_t> ess;
    build_essential(m->nx, m->ny, m->nz, sp->p, ess, sp->ess_mask);
  } catch (const std::bad_alloc&) {
    set_error("host memory exhausted building the integer maps");
    return PAFEM_ERR_OUT_OF_MEMORY;
  }
  sp->have_maps = true;
  return PAFEM_OK;
}

int ensure_device_maps(Space* sp) {
  if (sp->have_dev_maps) return PAFEM_OK;
  PAFEM_TRY(ensure_host_maps(sp));
  PAFEM_TRY(upload(sp->d_E, sp->E.data(), sp->E.size()));
  PAFEM_TRY(upload(sp->d_et_off, sp->et_off.data(), sp->et_off.size()));
  PAFEM_TRY(upload(sp->d_et_idx, sp->et_idx.data(), sp->et_idx.size()));
  PAFEM_TRY(upload(sp->d_ess_mask, sp->ess_mask.data(), sp->ess_mask.size()));
  sp->have_dev_maps = true;
  return PAFEM_OK;
}

// Ascending list of the boundary nodes of the lattice (surface only, so cheap).
int ensure_ess(Space* sp, bool device) {
  if (!sp->have_ess) {
    const int p = sp->p;
    const int64_t lx = (int64_t)sp->mesh->nx * p + 1, ly = (int64_t)sp->mesh->ny * p + 1,
                  lz = (int64_t)sp->mesh->nz * p + 1;
    sp->ess.clear();
    for (int64_t K = 0; K < lz; ++K)
      for (int64_t J = 0; J < ly; ++J) {
        const bool face = K == 0 || K == lz - 1 || J == 0 || J == ly - 1;
        if (face) {
          for (int64_t I = 0; I < lx; ++I) sp->ess.push_back((int32_t)(I + lx * (J + ly * K)));
        } else {
          sp->ess.push_back((int32_t)(lx * (J + ly * K)));
          sp->ess.push_back((int32_t)(lx - 1 + lx * (J + ly * K)));
        }
      }
    sp->have_ess = true;
  }
  if (device && !sp->have_dev_ess) {
    PAFEM_TRY(upload(sp->d_ess, sp->ess.data(), sp->ess.size()));
    sp->have_dev_ess = true;
  }
  return PAFEM_OK;
}

template <typename T>
ApplyArgs<T> make_args(Op* op, const T* x, T* y, T* yE, int flags, const int* skip,
                       int qprec = 0) {
  Space* sp = op->space;
  const int n = sp->p + 1;
  const DevBuf& tab = std::is_same<T, double>::value ? op->d_tab64 : op->d_tab32;
  ApplyArgs<T> a{};
  a.x = x;
  a.y = y;
  a.yE = yE;
  a.E = sp->d_E.as<int32_t>();
  a.ess_mask = sp->d_ess_mask.as<uint8_t>();
  a.qd = std::is_same<T, double>::value ? (const T*)op->d_qd64.ptr : (const T*)op->d_qd32.ptr;
  a.qd16 = (!std::is_same<T, double>::value && qprec == PAFEM_BF16) ? op->d_qd16.as<uint16_t>()
                                                                    : nullptr;
  if (a.qd16 != nullptr) a.qd = nullptr;
  a.B = tabB<T>(tab);
  a.G = tabG<T>(tab, op->q, n);
  a.ne = sp->ne;
  a.nx = sp->mesh->nx;
  a.ny = sp->mesh->ny;
  a.nz = sp->mesh->nz;
  a.constrained = (flags & PAFEM_APPLY_CONSTRAINED) ? 1 : 0;
  a.accumulate = (flags & PAFEM_APPLY_ACCUMULATE) ? 1 : 0;
  a.skip = skip;
  if (op->level == PAFEM_ASSEMBLY_MATRIX_FREE) {
    a.mf = 1;
    a.qd = nullptr;
    a.qd16 = nullptr;
    a.coef_kind = op->coef_kind;
    a.coef_value = op->coef_value;
    a.verts = sp->mesh->d_verts.as<double>();
    a.qpts = tabPts(op->d_tab64, op->q, n);
    a.qwts = tabWts(op->d_tab64, op->q, n);
  }
  return a;
}

template <typename T>
int apply_impl(Op* op, const T* x, T* y, int flags, const int* skip, hipStream_t s, int qprec,
               void* work) {
  Space* sp = op->space;
  const int n = sp->p + 1;
  if (work != nullptr) {
    // caller-provided E-vector workspace: the deterministic E^T on the
    // lattice numbering, nothing allocated (the maps are not needed)
    ApplyArgs<T> a = make_args<T>(op, x, y, static_cast<T*>(work), flags, skip, qprec);
    PAFEM_TRY_HIP(launch_apply<T>(op->kind, sp->p, op->q, kScatterXRows, PAFEM_INDEX_LATTICE, a, s));
    const bool tuned = op->level == PAFEM_ASSEMBLY_PARTIAL && op->q == sp->p + 2;
    const bool f64 = sizeof(T) == sizeof(double);
    PAFEM_TRY_HIP(launch_gather_xrows<T>(a.yE, a.nx, a.ny, a.nz, sp->p, a.constrained,
                                         a.accumulate, x, y, skip, s,
                                         tuned && evec_nt_loads(op->kind, sp->p, f64),
                                         tuned && y_nt_stores(op->kind, sp->p, f64)));
    return PAFEM_OK;
  }
  const int im = op->index_mode;
  if (im == PAFEM_INDEX_MAP) PAFEM_TRY(ensure_device_maps(sp));
  if (op->scatter_mode == PAFEM_SCATTER_ATOMIC && (flags & PAFEM_APPLY_CONSTRAINED))
    PAFEM_TRY(ensure_ess(sp, true));
  if (op->scatter_mode == PAFEM_SCATTER_DETERMINISTIC || op->level == PAFEM_ASSEMBLY_MATRIX_FREE) {
    if (op->level == PAFEM_ASSEMBLY_MATRIX_FREE) {
      PAFEM_TRY(op->d_evec.ensure((size_t)evec_words(sp->ne, n) * sizeof(double)));
      return apply_impl<T>(op, x, y, flags, skip, s, qprec, op->d_evec.ptr);
    }
    PAFEM_TRY(op->d_evec.ensure((size_t)evec_words(sp->ne, n) * sizeof(double)));
    if (im == PAFEM_INDEX_LATTICE)
      return apply_impl<T>(op, x, y, flags, skip, s, qprec, op->d_evec.ptr);
    // element pass into the E-vector, then the ordered per-node sum
    ApplyArgs<T> a = make_args<T>(op, x, y, op->d_evec.as<T>(), flags, skip, qprec);
    PAFEM_TRY_HIP(launch_apply<T>(op->kind, sp->p, op->q, kScatterEvector, im, a, s));
    PAFEM_TRY_HIP(launch_gather_et<T>(a.yE, sp->d_et_off.as<int32_t>(), sp->d_et_idx.as<int32_t>(),
                                      a.ess_mask, a.constrained, a.accumulate, x, y, sp->ndofs,
                                      skip, s));
  } else {
    ApplyArgs<T> a = make_args<T>(op, x, y, nullptr, flags, skip, qprec);
    // zero y with a kernel (not a memset) so the sequence can sit in a captured graph
    if (!a.accumulate) PAFEM_TRY_HIP(launch_fill<T>(y, sp->ndofs, T(0), skip, s));
    if (a.constrained)
      PAFEM_TRY_HIP(launch_set_ess<T>(sp->d_ess.as<int32_t>(), (int64_t)sp->ess.size(), x, T(0),
                                      a.accumulate, y, skip, s));
    PAFEM_TRY_HIP(launch_apply<T>(op->kind, sp->p, op->q, PAFEM_SCATTER_ATOMIC, im, a, s));
  }
  return PAFEM_OK;
}

template <typename T>
int apply_elements_dot(Op* op, const T* p, const int* skip, hipStream_t s, int qprec,
                       int* nparts) {
  Space* sp = op->space;
  if (op->scatter_mode != PAFEM_SCATTER_DETERMINISTIC || op->index_mode != PAFEM_INDEX_LATTICE) {
    set_error("internal: the fused CG element pass needs the lattice numbering");
    return PAFEM_ERR_INVALID_ARG;
  }
  const int64_t nb = element_blocks(op->kind, sp->p, sp->ne, !std::is_same<T, double>::value);
  if (nb <= 0 || nb > INT32_MAX) {
    set_error("internal: element workgroup count out of range");
    return PAFEM_ERR_INVALID_ARG;
  }
  PAFEM_TRY(op->d_evec.ensure((size_t)evec_words(sp->ne, sp->p + 1) * sizeof(double)));
  PAFEM_TRY(op->d_gpart.ensure((size_t)nb * sizeof(double)));
  ApplyArgs<T> a =
      make_args<T>(op, p, nullptr, op->d_evec.as<T>(), PAFEM_APPLY_CONSTRAINED, skip, qprec);
  a.dot_part = op->d_gpart.as<double>();
  PAFEM_TRY_HIP(
      launch_apply<T>(op->kind, sp->p, op->q, kScatterXRowsDot, PAFEM_INDEX_LATTICE, a, s));
  *nparts = (int)nb;
  return PAFEM_OK;
}
template int apply_elements_dot<double>(Op*, const double*, const int*, hipStream_t, int, int*);

int cg_element_args(Op* op, const double* p, ApplyArgs<double>* out, int64_t* groups) {
  Space* sp = op->space;
  const int64_t nb = element_blocks(op->kind, sp->p, sp->ne, false);
  if (nb <= 0 || nb > INT32_MAX) {
    set_error("internal: element workgroup count out of range");
    return PAFEM_ERR_INVALID_ARG;
  }
  PAFEM_TRY(op->d_evec.ensure((size_t)evec_words(sp->ne, sp->p + 1) * sizeof(double)));
  PAFEM_TRY(op->d_gpart.ensure((size_t)nb * sizeof(double)));
  *out = make_args<double>(op, p, nullptr, op->d_evec.as<double>(), PAFEM_APPLY_CONSTRAINED,
                           nullptr);
  out->dot_part = op->d_gpart.as<double>();
  *groups = nb;
  return PAFEM_OK;
}
template int apply_elements_dot<float>(Op*, const float*, const int*, hipStream_t, int, int*);

// y = E^T yE over every node (constrained: essential rows set to 0), in the
// op's restriction mode.
int gather_full(Op* op, const double* yE, int constrained, double* y, hipStream_t s) {
  Space* sp = op->space;
  if (op->index_mode == PAFEM_INDEX_MAP) {
    PAFEM_TRY(ensure_device_maps(sp));
    PAFEM_TRY_HIP(launch_gather_et<double>(yE, sp->d_et_off.as<int32_t>(),
                                           sp->d_et_idx.as<int32_t>(),
                                           sp->d_ess_mask.as<uint8_t>(), constrained, 0, nullptr,
                                           y, sp->ndofs, nullptr, s));
  } else {
    PAFEM_TRY_HIP(launch_gather_lattice<double>(yE, sp->mesh->nx, sp->mesh->ny, sp->mesh->nz,
                                                sp->p, constrained, 0, nullptr, y, nullptr, s));
  }
  return PAFEM_OK;
}

int diagonal_impl(Op* op, double* d, int constrained, hipStream_t s) {
  // element diagonals into the E-vector, then the ordered per-dof sum over all
  // nodes; essential rows are fixed up by the caller
  (void)constrained;
  Space* sp = op->space;
  const int n = sp->p + 1;
  PAFEM_TRY(op->d_evec.ensure((size_t)evec_words(sp->ne, n) * sizeof(double)));
  const double* qd = op->d_qd64.as<double>();
  DevBuf tmp;  // matrix-free: D computed for the diagonal only, then released
  if (op->level == PAFEM_ASSEMBLY_MATRIX_FREE) {
    const size_t nq = (size_t)sp->ne * op->q * op->q * op->q * op->ncomp;
    PAFEM_TRY(tmp.ensure(nq * sizeof(double)));
    GeomArgs g = geom(op, tabPts(op->d_tab64, op->q, n), tabWts(op->d_tab64, op->q, n));
    PAFEM_TRY_HIP(launch_qdata(g, op->kind, op->coef_kind, op->coef_value, nullptr,
                               tmp.as<double>(), nullptr, nullptr, op->d_flag.as<int>(), s));
    qd = tmp.as<double>();
  }
  PAFEM_TRY_HIP(launch_diag_elem(op->kind, sp->p, op->q, qd, tabB<double>(op->d_tab64),
                                 tabG<double>(op->d_tab64, op->q, n), sp->ne,
                                 op->d_evec.as<double>(), s));
  PAFEM_TRY(gather_full(op, op->d_evec.as<double>(), 0, d, s));
  if (tmp.ptr) PAFEM_TRY_HIP(hipStreamSynchronize(s));  // before the temporary is freed
  return PAFEM_OK;
}

template int apply_impl<double>(Op*, const double*, double*, int, const int*, hipStream_t, int,
                                void*);
template int apply_impl<float>(Op*, const float*, float*, int, const int*, hipStream_t, int,
                               void*);

}  // namespace pafem

using namespace pafem;


namespace {

void release(pafem_ctx* c) {
  if (c && --c->refs == 0) {
    if (!c->host_only) (void)hipSetDevice(c->device);
    delete c;
  }
}

void release(pafem_mesh* m) {
  if (m && --m->refs == 0) {
    auto* c = static_cast<pafem_ctx*>(m->ctx);
    if (!c->host_only) (void)hipSetDevice(c->device);
    delete m;
    release(c);
  }
}

void release(pafem_space* s) {
  if (s && --s->refs == 0) {
    auto* m = static_cast<pafem_mesh*>(s->mesh);
    if (!m->ctx->host_only) (void)hipSetDevice(m->ctx->device);
    delete s;
    release(m);
  }
}

void release(pafem_op* o) {
  if (o && --o->refs == 0) {
    auto* s = static_cast<pafem_space*>(o->space);
    (void)hipSetDevice(s->mesh->ctx->device);
    delete o;
    release(s);
  }
}

}  // namespace

extern "C" {

const char* pafem_last_error(void) { return g_err.c_str(); }

int pafem_version(void) { return 100; }

int pafem_ctx_create(int device, pafem_ctx** out) {
  clear_error();
  CHECK_ARG(out != nullptr, "out is NULL");
  *out = nullptr;
  CHECK_ARG(device >= -1, "device must be >= -1");
  auto* c = new pafem_ctx();
  c->device = device;
  c->host_only = device < 0;
  if (!c->host_only) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || device >= count) {
      delete c;
      set_error("HIP device " + std::to_string(device) + " not available (" +
                std::to_string(count) + " visible)");
      return PAFEM_ERR_NO_DEVICE;
    }
    e = hipSetDevice(device);
    if (e == hipSuccess) e = upload_basis_tables();
    if (e != hipSuccess) {
      delete c;
      set_error(std::string("device setup: ") + hipGetErrorString(e));
      return PAFEM_ERR_HIP;
    }
    const int rc = noalloc_init(device);
    if (rc != PAFEM_OK) {
      delete c;
      return rc;
    }
  }
  *out = c;
  return PAFEM_OK;
}

int pafem_ctx_destroy(pafem_ctx* ctx) {
  release(ctx);
  return PAFEM_OK;
}

int pafem_mesh_create_structured(pafem_ctx* ctx, int nx, int ny, int nz,
                                 const double* vert_xyz_host, pafem_mesh** out) {
  clear_error();
  CHECK_ARG(ctx && out && vert_xyz_host, "NULL argument");
  *out = nullptr;
  CHECK_ARG(nx >= 1 && ny >= 1 && nz >= 1, "nx, ny, nz must be >= 1");
  const int64_t nv = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  CHECK_ARG((int64_t)nx * ny * nz < std::numeric_limits<int32_t>::max(), "too many elements");
  for (int64_t i = 0; i < nv * 3; ++i)
    CHECK_ARG(std::isfinite(vert_xyz_host[i]), "vertex coordinates must be finite");
  auto* m = new pafem_mesh();
  m->ctx = ctx;
  m->nx = nx;
  m->ny = ny;
  m->nz = nz;
  m->verts.assign(vert_xyz_host, vert_xyz_host + nv * 3);
  if (!ctx->host_only) {
    int rc = need_device(ctx);
    if (rc == PAFEM_OK) rc = upload(m->d_verts, m->verts.data(), m->verts.size());
    if (rc != PAFEM_OK) {
      delete m;
      return rc;
    }
  }
  ++ctx->refs;
  *out = m;
  return PAFEM_OK;
}

int pafem_mesh_destroy(pafem_mesh* mesh) {
  release(mesh);
  return PAFEM_OK;
}

int pafem_space_create(pafem_mesh* mesh, int p, pafem_space** out) {
  clear_error();
  CHECK_ARG(mesh && out, "NULL argument");
  *out = nullptr;
  CHECK_ARG(p >= 1 && p <= kMaxP, "p must be in 1..8");
  const int64_t n = p + 1;
  const int64_t ne = (int64_t)mesh->nx * mesh->ny * mesh->nz;
  const int64_t ndofs =
      ((int64_t)mesh->nx * p + 1) * ((int64_t)mesh->ny * p + 1) * ((int64_t)mesh->nz * p + 1);
  CHECK_ARG(evec_words(ne, (int)n) < std::numeric_limits<int32_t>::max(),
            "the E-vector (about ne*(p+1)^3 words) must fit in int32 indexing");
  CHECK_ARG(ndofs < std::numeric_limits<int32_t>::max(), "ndofs must fit in int32");
  auto* sp = new pafem_space();
  sp->mesh = mesh;
  sp->p = p;
  sp->ne = ne;
  sp->ndofs = ndofs;
  if (!mesh->ctx->host_only) {
    int rc = need_device(mesh->ctx);
    if (rc != PAFEM_OK) {
      delete sp;
      return rc;
    }
  }
  ++mesh->refs;
  *out = sp;
  return PAFEM_OK;
}

int pafem_space_destroy(pafem_space* space) {
  release(space);
  return PAFEM_OK;
}

int64_t pafem_space_ndofs(const pafem_space* s) { return s ? s->ndofs : -1; }
int64_t pafem_space_nelems(const pafem_space* s) { return s ? s->ne : -1; }
int64_t pafem_space_num_ess(const pafem_space* s) {
  if (!s) return -1;
  const int64_t lx = (int64_t)s->mesh->nx * s->p + 1, ly = (int64_t)s->mesh->ny * s->p + 1,
                lz = (int64_t)s->mesh->nz * s->p + 1;
  return lx * ly * lz - (lx - 2) * (ly - 2) * (lz - 2);
}

int pafem_space_get_restriction(const pafem_space* s, int32_t* E_host) {
  clear_error();
  CHECK_ARG(s && E_host, "NULL argument");
  PAFEM_TRY(ensure_host_maps(const_cast<pafem_space*>(s)));
  std::memcpy(E_host, s->E.data(), s->E.size() * sizeof(int32_t));
  return PAFEM_OK;
}

int pafem_space_get_restriction_transpose(const pafem_space* s, int32_t* off, int32_t* idx) {
  clear_error();
  CHECK_ARG(s && off && idx, "NULL argument");
  PAFEM_TRY(ensure_host_maps(const_cast<pafem_space*>(s)));
  std::memcpy(off, s->et_off.data(), s->et_off.size() * sizeof(int32_t));
  std::memcpy(idx, s->et_idx.data(), s->et_idx.size() * sizeof(int32_t));
  return PAFEM_OK;
}

int pafem_space_get_ess_dofs(const pafem_space* s, int32_t* out) {
  clear_error();
  CHECK_ARG(s && out, "NULL argument");
  PAFEM_TRY(ensure_ess(const_cast<pafem_space*>(s), false));
  std::memcpy(out, s->ess.data(), s->ess.size() * sizeof(int32_t));
  return PAFEM_OK;
}

int pafem_basis_tables(int p, int q, double* nodes, double* pts, double* wts, double* B,
                       double* G) {
  clear_error();
  CHECK_ARG(p >= 1 && p <= kMaxP, "p must be in 1..8");
  CHECK_ARG(q >= 1 && q <= kMaxQ, "q must be in 1..12");
  std::vector<double> nd(p + 1), x(q), w(q), b(q * (p + 1)), g(q * (p + 1));
  gll_nodes(p, nd.data());
  gauss_legendre(q, x.data(), w.data());
  lagrange_tables(p + 1, nd.data(), q, x.data(), b.data(), g.data());
  if (nodes) std::memcpy(nodes, nd.data(), nd.size() * sizeof(double));
  if (pts) std::memcpy(pts, x.data(), x.size() * sizeof(double));
  if (wts) std::memcpy(wts, w.data(), w.size() * sizeof(double));
  if (B) std::memcpy(B, b.data(), b.size() * sizeof(double));
  if (G) std::memcpy(G, g.data(), g.size() * sizeof(double));
  return PAFEM_OK;
}

int pafem_op_create(pafem_space* space, int kind, int q1d, pafem_op** out) {
  clear_error();
  CHECK_ARG(space && out, "NULL argument");
  *out = nullptr;
  CHECK_ARG(kind == PAFEM_MASS || kind == PAFEM_DIFFUSION, "kind must be MASS or DIFFUSION");
  const int p = space->p;
  const int q = q1d == 0 ? p + 2 : q1d;
  if (q < p + 1 || q > kMaxQ1d) {
    set_error("q1d must be 0 (p + 2) or within p + 1 .. 10");
    return PAFEM_ERR_UNSUPPORTED;
  }
  PAFEM_TRY(need_device(space->mesh->ctx));
  auto* op = new pafem_op();
  op->space = space;
  op->kind = kind;
  op->q = q;
  op->ncomp = kind == PAFEM_DIFFUSION ? 6 : 1;
  const int n = p + 1;
  std::vector<double> nd(n), x(q), w(q), tab(2 * q * n + 2 * q);
  gll_nodes(p, nd.data());
  gauss_legendre(q, x.data(), w.data());
  lagrange_tables(n, nd.data(), q, x.data(), tab.data(), tab.data() + q * n);
  std::memcpy(tab.data() + 2 * q * n, x.data(), q * sizeof(double));
  std::memcpy(tab.data() + 2 * q * n + q, w.data(), q * sizeof(double));
  std::vector<float> tab32(tab.size());
  for (size_t i = 0; i < tab.size(); ++i) tab32[i] = (float)tab[i];
  int rc = upload(op->d_tab64, tab.data(), tab.size());
  if (rc == PAFEM_OK) rc = upload(op->d_tab32, tab32.data(), tab32.size());
  if (rc == PAFEM_OK) rc = op->d_flag.ensure(sizeof(int));
  if (rc != PAFEM_OK) {
    delete op;
    return rc;
  }
  ++space->refs;
  *out = op;
  return PAFEM_OK;
}

int pafem_op_destroy(pafem_op* op) {
  release(op);
  return PAFEM_OK;
}

int pafem_op_q1d(const pafem_op* op) { return op ? op->q : -1; }

int pafem_op_qpoint_coords(pafem_op* op, double* xyz, void* stream) {
  clear_error();
  CHECK_ARG(op && xyz, "NULL argument");
  PAFEM_TRY(need_device(op->space->mesh->ctx));
  const int n = op->space->p + 1;
  GeomArgs g = geom(op, tabPts(op->d_tab64, op->q, n), tabWts(op->d_tab64, op->q, n));
  PAFEM_TRY_HIP(launch_qpoint_coords(g, xyz, S(stream)));
  return PAFEM_OK;
}

int pafem_op_set_coefficient_const(pafem_op* op, double c) {
  clear_error();
  CHECK_ARG(op, "NULL argument");
  CHECK_ARG(std::isfinite(c), "coefficient must be finite");
  op->coef_kind = COEF_CONST;
  op->coef_value = c;
  return PAFEM_OK;
}

int pafem_op_set_coefficient_qpts(pafem_op* op, const double* k, void* stream) {
  clear_error();
  CHECK_ARG(op && k, "NULL argument");
  PAFEM_TRY(need_device(op->space->mesh->ctx));
  const size_t n = (size_t)op->space->ne * op->q * op->q * op->q;
  PAFEM_TRY(op->d_coef.ensure(n * sizeof(double)));
  PAFEM_TRY_HIP(hipMemcpyAsync(op->d_coef.ptr, k, n * sizeof(double), hipMemcpyDeviceToDevice,
                               S(stream)));
  op->coef_kind = COEF_QPTS;
  return PAFEM_OK;
}

int pafem_op_set_coefficient_sinx(pafem_op* op, double amp) {
  clear_error();
  CHECK_ARG(op, "NULL argument");
  CHECK_ARG(std::isfinite(amp), "amplitude must be finite");
  op->coef_kind = COEF_SINX;
  op->coef_value = amp;
  return PAFEM_OK;
}

int64_t pafem_op_qdata_bytes(const pafem_op* op, int prec_mask) {
  if (!op) return -1;
  if (op->level == PAFEM_ASSEMBLY_MATRIX_FREE) return 0;
  const int64_t n = op->space->ne * (int64_t)op->q * op->q * op->q * op->ncomp;
  int64_t b = n * 8;
  if (prec_mask & PAFEM_FP32) b += n * 4;
  if (prec_mask & PAFEM_BF16) b += n * 2;
  return b;
}

int64_t pafem_op_footprint_bytes(const pafem_op* op, int prec_mask) {
  if (!op || (prec_mask & ~(PAFEM_FP64 | PAFEM_FP32 | PAFEM_BF16)) != 0) return -1;
  const Space* sp = op->space;
  const int64_t n = sp->ndofs;
  const bool f32 = (prec_mask & (PAFEM_FP32 | PAFEM_BF16)) != 0;
  int64_t b = pafem_op_qdata_bytes(op, prec_mask | PAFEM_FP64);
  b += evec_words(sp->ne, sp->p + 1) * 8;        // E-vector workspace
  b += n * (8 + (f32 ? 4 : 0));                   // inverse diagonal
  b += n * (3 * 8 + 8) + (f32 ? n * 4 * 4 : 0);   // CG vectors (+ x for the graph form)
  const int64_t nb = reduce_blocks(n);
  b += ((nb > kMaxCgParts ? nb : kMaxCgParts) * 2 + 8) * 8;  // reduction partials
  b += element_blocks(op->kind, sp->p, sp->ne, false) * 8;  // element-pass partials
  return b;
}

int pafem_op_assemble(pafem_op* op, int prec_mask, void* stream) {
  clear_error();
  CHECK_ARG(op, "NULL argument");
  CHECK_ARG((prec_mask & ~(PAFEM_FP64 | PAFEM_FP32 | PAFEM_BF16)) == 0, "unknown precision bits");
  PAFEM_TRY(need_device(op->space->mesh->ctx));
  const bool mf = op->level == PAFEM_ASSEMBLY_MATRIX_FREE;
  if ((prec_mask & PAFEM_BF16) && op->q != op->space->p + 2) {
    set_error("bfloat16 quadrature data needs the default q1d = p + 2");
    return PAFEM_ERR_UNSUPPORTED;
  }
  if (mf) {
    CHECK_ARG((prec_mask & PAFEM_BF16) == 0,
              "a matrix-free operator stores no quadrature data to round to bfloat16");
    CHECK_ARG(op->coef_kind != COEF_QPTS,
              "a matrix-free operator needs a constant or the built-in coefficient");
  }
  const size_t n = (size_t)op->space->ne * op->q * op->q * op->q * op->ncomp;
  if (!mf) PAFEM_TRY(op->d_qd64.ensure(n * sizeof(double)));
  float* q32 = nullptr;
  if ((prec_mask & PAFEM_FP32) && !mf) {
    PAFEM_TRY(op->d_qd32.ensure(n * sizeof(float)));
    q32 = op->d_qd32.as<float>();
  }
  uint16_t* q16 = nullptr;
  if (prec_mask & PAFEM_BF16) {
    PAFEM_TRY(op->d_qd16.ensure(n * sizeof(uint16_t)));
    q16 = op->d_qd16.as<uint16_t>();
  }
  const int nn = op->space->p + 1;
  GeomArgs g = geom(op, tabPts(op->d_tab64, op->q, nn), tabWts(op->d_tab64, op->q, nn));
  hipStream_t s = S(stream);
  PAFEM_TRY_HIP(hipMemsetAsync(op->d_flag.ptr, 0, sizeof(int), s));
  // (matrix-free: the same pass with nothing stored checks the Jacobian sign)
  PAFEM_TRY_HIP(launch_qdata(g, op->kind, op->coef_kind, op->coef_value, op->d_coef.as<double>(),
                             mf ? nullptr : op->d_qd64.as<double>(), q32, q16,
                             op->d_flag.as<int>(), s));
  int flag = 0;
  PAFEM_TRY_HIP(hipMemcpyAsync(&flag, op->d_flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
  PAFEM_TRY_HIP(hipStreamSynchronize(s));
  op->have64 = true;
  op->have32 = mf ? (prec_mask & PAFEM_FP32) != 0 : q32 != nullptr;
  op->have16 = q16 != nullptr;
  op->have_dinv = false;
  if (flag) {
    op->have64 = op->have32 = op->have16 = false;
    set_error("non-positive Jacobian determinant at a quadrature point (inverted element)");
    return PAFEM_ERR_INVALID_ARG;
  }
  return PAFEM_OK;
}

int pafem_op_get_qdata(pafem_op* op, int prec, void* dst, void* stream) {
  clear_error();
  CHECK_ARG(op && dst, "NULL argument");
  CHECK_ARG(op->level == PAFEM_ASSEMBLY_PARTIAL, "a matrix-free operator stores no quadrature data");
  CHECK_ARG(prec == PAFEM_FP64 || prec == PAFEM_FP32 || prec == PAFEM_BF16,
            "prec must be FP64, FP32 or BF16");
  const bool have = prec == PAFEM_FP64 ? op->have64 : prec == PAFEM_FP32 ? op->have32 : op->have16;
  CHECK_ARG(have, "quadrature data of that precision not assembled");
  const size_t n = (size_t)op->space->ne * op->q * op->q * op->q * op->ncomp;
  const void* src = prec == PAFEM_FP64 ? op->d_qd64.ptr
                    : prec == PAFEM_FP32 ? op->d_qd32.ptr : op->d_qd16.ptr;
  const size_t bytes = prec == PAFEM_FP64 ? 8 : prec == PAFEM_FP32 ? 4 : 2;
  PAFEM_TRY_HIP(hipMemcpyAsync(dst, src, n * bytes, hipMemcpyDeviceToDevice, S(stream)));
  return PAFEM_OK;
}

int pafem_op_set_assembly_level(pafem_op* op, int level) {
  clear_error();
  CHECK_ARG(op, "NULL argument");
  CHECK_ARG(level == PAFEM_ASSEMBLY_PARTIAL || level == PAFEM_ASSEMBLY_MATRIX_FREE,
            "unknown assembly level");
  if (level == PAFEM_ASSEMBLY_MATRIX_FREE) {
    CHECK_ARG(op->scatter_mode == PAFEM_SCATTER_DETERMINISTIC &&
                  op->index_mode == PAFEM_INDEX_LATTICE,
              "the matrix-free level runs the deterministic E^T on the lattice numbering");
    if (op->q != op->space->p + 2) {
      set_error("the matrix-free level needs the default q1d = p + 2");
      return PAFEM_ERR_UNSUPPORTED;
    }
  }
  if (level != op->level) {
    op->level = level;
    op->have64 = op->have32 = op->have16 = false;
    op->have_dinv = false;
    op->d_qd64.release();
    op->d_qd32.release();
    op->d_qd16.release();
  }
  return PAFEM_OK;
}

int pafem_op_set_scatter_mode(pafem_op* op, int mode) {
  clear_error();
  CHECK_ARG(op, "NULL argument");
  CHECK_ARG(mode == PAFEM_SCATTER_ATOMIC || mode == PAFEM_SCATTER_DETERMINISTIC,
            "unknown scatter mode");
  CHECK_ARG(op->level == PAFEM_ASSEMBLY_PARTIAL || mode == PAFEM_SCATTER_DETERMINISTIC,
            "the matrix-free level runs the deterministic E^T");
  op->scatter_mode = mode;
  return PAFEM_OK;
}

int pafem_op_set_restriction_mode(pafem_op* op, int mode) {
  clear_error();
  CHECK_ARG(op, "NULL argument");
  CHECK_ARG(mode == PAFEM_INDEX_LATTICE || mode == PAFEM_INDEX_MAP, "unknown restriction mode");
  CHECK_ARG(op->level == PAFEM_ASSEMBLY_PARTIAL || mode == PAFEM_INDEX_LATTICE,
            "the matrix-free level runs on the lattice numbering");
  op->index_mode = mode;
  return PAFEM_OK;
}

int pafem_op_apply(pafem_op* op, int prec, const void* x, void* y, int flags, void* stream) {
  clear_error();
  CHECK_ARG(op && x && y, "NULL argument");
  CHECK_ARG(x != y, "x and y must not alias");
  CHECK_ARG((flags & ~(PAFEM_APPLY_CONSTRAINED | PAFEM_APPLY_ACCUMULATE)) == 0,
            "unknown apply flags");
  PAFEM_TRY(need_device(op->space->mesh->ctx));
  if (prec == PAFEM_FP64) {
    CHECK_ARG(op->have64, "operator not assembled");
    return apply_impl<double>(op, (const double*)x, (double*)y, flags, nullptr, S(stream));
  }
  if (prec == PAFEM_FP32) {
    CHECK_ARG(op->have32, "FP32 quadrature data not assembled");
    return apply_impl<float>(op, (const float*)x, (float*)y, flags, nullptr, S(stream));
  }
  if (prec == PAFEM_BF16) {
    CHECK_ARG(op->have16, "BF16 quadrature data not assembled");
    return apply_impl<float>(op, (const float*)x, (float*)y, flags, nullptr, S(stream),
                             PAFEM_BF16);
  }
  set_error("prec must be PAFEM_FP64, PAFEM_FP32 or PAFEM_BF16");
  return PAFEM_ERR_INVALID_ARG;
}

int pafem_op_apply_evector(pafem_op* op, int prec, const void* x, void* yE, int flags,
                           void* stream) {
  clear_error();
  CHECK_ARG(op && x && yE, "NULL argument");
  CHECK_ARG(x != yE, "x and yE must not alias");
  CHECK_ARG((flags & ~PAFEM_APPLY_CONSTRAINED) == 0, "only PAFEM_APPLY_CONSTRAINED is allowed");
  PAFEM_TRY(need_device(op->space->mesh->ctx));
  Space* sp = op->space;
  hipStream_t s = S(stream);
  if (op->index_mode == PAFEM_INDEX_MAP) PAFEM_TRY(ensure_device_maps(sp));
  if (prec == PAFEM_FP64) {
    CHECK_ARG(op->have64, "operator not assembled");
    ApplyArgs<double> a = make_args<double>(op, (const double*)x, nullptr, (double*)yE, flags,
                                            nullptr);
    PAFEM_TRY_HIP(launch_apply<double>(op->kind, sp->p, op->q, kScatterEvector, op->index_mode, a, s));
    return PAFEM_OK;
  }
  if (prec == PAFEM_FP32 || prec == PAFEM_BF16) {
    CHECK_ARG(prec == PAFEM_FP32 ? op->have32 : op->have16,
              "quadrature data of that precision not assembled");
    ApplyArgs<float> a = make_args<float>(op, (const float*)x, nullptr, (float*)yE, flags, nullptr,
                                          prec);
    PAFEM_TRY_HIP(launch_apply<float>(op->kind, sp->p, op->q, kScatterEvector, op->index_mode, a, s));
    return PAFEM_OK;
  }
  set_error("prec must be PAFEM_FP64 or PAFEM_FP32");
  return PAFEM_ERR_INVALID_ARG;
}

int pafem_op_diagonal(pafem_op* op, double* d, int constrained, void* stream) {
  clear_error();
  CHECK_ARG(op && d, "NULL argument");
  CHECK_ARG(constrained == 0 || constrained == 1, "constrained must be 0 or 1");
  CHECK_ARG(op->have64, "operator not assembled");
  PAFEM_TRY(need_device(op->space->mesh->ctx));
  hipStream_t s = S(stream);
  PAFEM_TRY(diagonal_impl(op, d, constrained, s));
  if (constrained) {
    PAFEM_TRY(ensure_ess(op->space, true));
    PAFEM_TRY_HIP(launch_set_ess<double>(op->space->d_ess.as<int32_t>(),
                                         (int64_t)op->space->ess.size(), nullptr, 1.0, 0, d,
                                         nullptr, s));
  }
  return PAFEM_OK;
}

int pafem_rhs_assemble(pafem_op* op, const double* f_q, double* b, void* stream) {
  clear_error();
  CHECK_ARG(op && b, "NULL argument");
  PAFEM_TRY(need_device(op->space->mesh->ctx));
  Space* sp = op->space;
  const int n = sp->p + 1;
  PAFEM_TRY(op->d_evec.ensure((size_t)evec_words(sp->ne, n) * sizeof(double)));
  GeomArgs g = geom(op, tabPts(op->d_tab64, op->q, n), tabWts(op->d_tab64, op->q, n));
  hipStream_t s = S(stream);
  PAFEM_TRY_HIP(launch_rhs_elem(g, sp->p, tabB<double>(op->d_tab64), f_q, op->d_evec.as<double>(), s));
  return gather_full(op, op->d_evec.as<double>(), 1, b, s);
}

int pafem_dot(pafem_ctx* ctx, int64_t n, const double* x, const double* y, double* result,
              void* stream) {
  clear_error();
  CHECK_ARG(ctx && result && (n == 0 || (x && y)), "NULL argument");
  CHECK_ARG(n >= 0, "n must be >= 0");
  PAFEM_TRY(need_device(ctx));
  const int nb = reduce_blocks(n);
  PAFEM_TRY(ctx->scratch.ensure(nb * sizeof(double)));
  hipStream_t s = S(stream);
  PAFEM_TRY_HIP(launch_dot_partial<double>(x, y, n, ctx->scratch.as<double>(), nb, nullptr, s));
  PAFEM_TRY_HIP(launch_sum_final(ctx->scratch.as<double>(), nb, 1, result, s));
  return PAFEM_OK;
}

}  // extern "C"
