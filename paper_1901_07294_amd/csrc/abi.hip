// C entry points of wilson.h: argument checks, handles, dispatch to kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "eo.h"
#include "fields.h"
#include "wd_internal.h"

namespace wd {

namespace {
thread_local char g_last_error[512] = "";
}

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_last_error[0] = '\0'; }

size_t spinor_site_bytes(int prec) {
  switch (prec) {
    case WD_FP64: return 24 * sizeof(double);
    case WD_FP32: return 24 * sizeof(float);
    case WD_FP16: return 24 * 2 + sizeof(float);  // binary16 components + per-site scale
    default: return 0;
  }
}

size_t gauge_site_bytes(int prec, int c12) {
  const size_t reals = 4 * (c12 ? 12 : 18);
  switch (prec) {
    case WD_FP64: return reals * sizeof(double);
    case WD_FP32: return reals * sizeof(float);
    case WD_FP16: return reals * 2;
    default: return 0;
  }
}

constexpr long kMaxSites = (1L << 31) / 12 - 1;  // keeps plane offsets in range

// Validates dims; on success stores the volume in *V.
int check_dims(const int32_t dims[4], long* V) {
  if (dims == nullptr) return set_error(WD_ERR_INVALID_ARG, "dims is NULL");
  long v = 1;
  for (int i = 0; i < 4; ++i) {
    if (dims[i] < 1)
      return set_error(WD_ERR_SHAPE, "lattice extent %d is %d; every extent must be >= 1", i,
                       dims[i]);
    v *= dims[i];
    if (v > kMaxSites) return set_error(WD_ERR_SHAPE, "lattice volume exceeds %ld sites", kMaxSites);
  }
  *V = v;
  return WD_OK;
}

int check_prec(int prec) {
  if (prec == WD_FP64 || prec == WD_FP32 || prec == WD_FP16) return WD_OK;
  return set_error(WD_ERR_INVALID_ARG, "unknown precision %d", prec);
}

// The range [p, p + bytes) must lie inside one device allocation on the
// current device.
int check_device_range(const void* p, size_t bytes, const char* what) {
  if (p == nullptr) return set_error(WD_ERR_INVALID_ARG, "%s is NULL", what);
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(WD_ERR_INVALID_ARG, "%s (%p) is not a HIP device pointer", what, p);
  }
  if (attr.type != hipMemoryTypeDevice)
    return set_error(WD_ERR_INVALID_ARG, "%s (%p) is not device memory (memory type %d)", what, p,
                     static_cast<int>(attr.type));
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != attr.device)
    return set_error(WD_ERR_INVALID_ARG, "%s lives on device %d, current device is %d", what,
                     attr.device, dev);
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(WD_ERR_INVALID_ARG, "%s (%p): cannot query its allocation", what, p);
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(p);
  if (q < b || static_cast<size_t>(q - b) + bytes > size)
    return set_error(WD_ERR_INVALID_ARG,
                     "%s (%p) needs %zu bytes but its allocation ends %zu bytes after it", what, p,
                     bytes, static_cast<size_t>(b + size - q));
  return WD_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + nb && y < x + na;
}

int check_gauge(const wd_gauge* g) {
  if (g == nullptr) return set_error(WD_ERR_INVALID_ARG, "gauge handle is NULL");
  if (g->magic != kGaugeMagic) return set_error(WD_ERR_INVALID_ARG, "not a live gauge handle");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != g->device)
    return set_error(WD_ERR_INVALID_ARG, "gauge handle belongs to device %d, current device is %d",
                     g->device, dev);
  return WD_OK;
}

// g must have the full-lattice layout (eo == 0) or the even-odd one (eo == 1).
int check_layout(const wd_gauge* g, int eo, const char* what) {
  if (g->eo == eo) return WD_OK;
  return set_error(WD_ERR_INVALID_ARG, eo ? "%s needs an even-odd gauge handle (wd_gauge_import_eo)"
                                          : "%s needs a full-lattice gauge handle (wd_gauge_import)",
                   what);
}

int check_even_dims(const int32_t dims[4]) {
  for (int i = 0; i < 4; ++i)
    if (dims[i] % 2 != 0)
      return set_error(WD_ERR_SHAPE, "even-odd layout needs even extents; extent %d is %d", i, dims[i]);
  return WD_OK;
}

int launch_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return WD_OK;
  return set_error(WD_ERR_DEVICE, "%s: launch failed: %s", what, hipGetErrorString(e));
}

}  // namespace wd

using namespace wd;

extern "C" {

int wd_abi_version(void) { return WD_ABI_VERSION; }

const char* wd_last_error(void) { return g_last_error; }

size_t wd_spinor_bytes(const int32_t dims[4], int32_t prec, int32_t nrhs) {
  long V = 0;
  if (check_dims(dims, &V) != WD_OK || nrhs < 0) return 0;
  return static_cast<size_t>(packed_sites(V)) * static_cast<size_t>(nrhs) * spinor_site_bytes(prec);
}

size_t wd_gauge_bytes(const int32_t dims[4], int32_t prec, int32_t compress12) {
  long V = 0;
  if (check_dims(dims, &V) != WD_OK) return 0;
  return static_cast<size_t>(packed_sites(V)) * gauge_site_bytes(prec, compress12 ? 1 : 0);
}

int wd_gauge_import(const int32_t dims[4], const void* U_canon_dev, int32_t prec,
                    int32_t compress12, void* dst_dev, size_t dst_bytes, hipStream_t stream,
                    wd_gauge** out) {
  try {
    clear_error();
    if (out == nullptr) return set_error(WD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    long V = 0;
    int rc = check_dims(dims, &V);
    if (rc != WD_OK) return rc;
    if ((rc = check_prec(prec)) != WD_OK) return rc;
    const int c12 = compress12 ? 1 : 0;
    const size_t need = static_cast<size_t>(packed_sites(V)) * gauge_site_bytes(prec, c12);
    if (dst_bytes < need)
      return set_error(WD_ERR_INVALID_ARG, "dst_bytes %zu < %zu needed", dst_bytes, need);
    const size_t canon_bytes = static_cast<size_t>(V) * 36 * 16;
    if ((rc = check_device_range(U_canon_dev, canon_bytes, "U_canon_dev")) != WD_OK) return rc;
    if ((rc = check_device_range(dst_dev, need, "dst_dev")) != WD_OK) return rc;
    if (overlaps(U_canon_dev, canon_bytes, dst_dev, need))
      return set_error(WD_ERR_INVALID_ARG, "U_canon_dev and dst_dev overlap");
    wd_gauge* g = new (std::nothrow) wd_gauge;
    if (g == nullptr) return set_error(WD_ERR_NOMEM, "host allocation of the handle failed");
    g->magic = kGaugeMagic;
    for (int i = 0; i < 4; ++i) g->dims[i] = dims[i];
    g->V = V;
    g->prec = prec;
    g->c12 = c12;
    g->eo = 0;
    (void)hipGetDevice(&g->device);
    g->links = dst_dev;
    g->link_bytes = need;
    rc = launch_status(launch_pack_gauge(U_canon_dev, dst_dev, make_geo(dims), prec, c12, stream),
                       "pack_gauge");
    if (rc != WD_OK) {
      g->magic = 0;
      delete g;
      return rc;
    }
    *out = g;
    return WD_OK;
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in wd_gauge_import");
  }
}

int wd_gauge_release(wd_gauge* g) {
  clear_error();
  if (g == nullptr) return WD_OK;
  if (g->magic != kGaugeMagic) return set_error(WD_ERR_INVALID_ARG, "not a live gauge handle");
  g->magic = 0;
  delete g;
  return WD_OK;
}

static int spinor_transfer(const wd_gauge* g, const void* src, int32_t prec, int32_t nrhs, void* dst,
                           hipStream_t stream, bool import) {
  int rc = check_gauge(g);
  if (rc != WD_OK) return rc;
  if ((rc = check_prec(prec)) != WD_OK) return rc;
  if (prec != g->prec)
    return set_error(WD_ERR_INVALID_ARG, "spinor precision %d differs from the gauge field's %d",
                     prec, g->prec);
  if (nrhs < 0) return set_error(WD_ERR_INVALID_ARG, "nrhs is %d", nrhs);
  if (nrhs == 0) return WD_OK;
  const size_t canon = static_cast<size_t>(g->V) * nrhs * 12 * 16;
  const size_t packed = static_cast<size_t>(packed_sites(g->V)) * nrhs * spinor_site_bytes(prec);
  const size_t nsrc = import ? canon : packed;
  const size_t ndst = import ? packed : canon;
  if ((rc = check_device_range(src, nsrc, import ? "canon_dev" : "src_dev")) != WD_OK) return rc;
  if ((rc = check_device_range(dst, ndst, import ? "dst_dev" : "canon_dev")) != WD_OK) return rc;
  if (overlaps(src, nsrc, dst, ndst)) return set_error(WD_ERR_INVALID_ARG, "buffers overlap");
  const Geo geo = make_geo(g->dims);
  return launch_status(import ? launch_pack_spinor(src, dst, geo, prec, nrhs, stream)
                              : launch_unpack_spinor(src, dst, geo, prec, nrhs, stream),
                       import ? "pack_spinor" : "unpack_spinor");
}

int wd_spinor_import(const wd_gauge* g, const void* canon_dev, int32_t prec, int32_t nrhs,
                     void* dst_dev, hipStream_t stream) {
  try {
    clear_error();
    return spinor_transfer(g, canon_dev, prec, nrhs, dst_dev, stream, true);
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in wd_spinor_import");
  }
}

int wd_spinor_export(const wd_gauge* g, const void* src_dev, int32_t prec, int32_t nrhs,
                     void* canon_dev, hipStream_t stream) {
  try {
    clear_error();
    return spinor_transfer(g, src_dev, prec, nrhs, canon_dev, stream, false);
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in wd_spinor_export");
  }
}

int dslash_apply(const wd_gauge* g, double mass, const void* in_dev, void* out_dev, int32_t prec,
                 int32_t flags, hipStream_t stream) {
  try {
    clear_error();
    int rc = check_gauge(g);
    if (rc != WD_OK) return rc;
    if ((rc = check_layout(g, 0, "dslash_apply")) != WD_OK) return rc;
    if ((rc = check_prec(prec)) != WD_OK) return rc;
    if (prec != g->prec)
      return set_error(WD_ERR_INVALID_ARG, "spinor precision %d differs from the gauge field's %d",
                       prec, g->prec);
    if (flags & ~WD_FLAG_GAMMA5) return set_error(WD_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const size_t n = static_cast<size_t>(packed_sites(g->V)) * spinor_site_bytes(prec);
    if ((rc = check_device_range(in_dev, n, "in_dev")) != WD_OK) return rc;
    if ((rc = check_device_range(out_dev, n, "out_dev")) != WD_OK) return rc;
    if (overlaps(in_dev, n, out_dev, n)) return set_error(WD_ERR_INVALID_ARG, "in_dev and out_dev overlap");
    return launch_status(launch_dslash(g, mass, in_dev, out_dev, flags, stream), "dslash");
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in dslash_apply");
  }
}

int dslash_apply_multi(const wd_gauge* g, const double* masses_host, int32_t nrhs,
                       const void* in_dev, void* out_dev, int32_t prec, int32_t flags,
                       hipStream_t stream) {
  try {
    clear_error();
    int rc = check_gauge(g);
    if (rc != WD_OK) return rc;
    if ((rc = check_layout(g, 0, "dslash_apply_multi")) != WD_OK) return rc;
    if ((rc = check_prec(prec)) != WD_OK) return rc;
    if (prec != g->prec)
      return set_error(WD_ERR_INVALID_ARG, "spinor precision %d differs from the gauge field's %d",
                       prec, g->prec);
    if (flags & ~WD_FLAG_GAMMA5) return set_error(WD_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (nrhs < 0) return set_error(WD_ERR_INVALID_ARG, "nrhs is %d", nrhs);
    if (nrhs > kMaxMultiRhs)
      return set_error(WD_ERR_UNSUPPORTED, "nrhs %d exceeds %d per launch", nrhs, kMaxMultiRhs);
    if (nrhs == 0) return WD_OK;
    if (masses_host == nullptr) return set_error(WD_ERR_INVALID_ARG, "masses_host is NULL");
    for (int k = 0; k < nrhs; ++k)
      if (!std::isfinite(masses_host[k])) return set_error(WD_ERR_INVALID_ARG, "mass %d is not finite", k);
    const size_t n = static_cast<size_t>(packed_sites(g->V)) * nrhs * spinor_site_bytes(prec);
    if ((rc = check_device_range(in_dev, n, "in_dev")) != WD_OK) return rc;
    if ((rc = check_device_range(out_dev, n, "out_dev")) != WD_OK) return rc;
    if (overlaps(in_dev, n, out_dev, n)) return set_error(WD_ERR_INVALID_ARG, "in_dev and out_dev overlap");
    return launch_status(launch_dslash_multi(g, masses_host, nrhs, nullptr, in_dev, out_dev, flags,
                                             stream), "dslash_multi");
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in dslash_apply_multi");
  }
}

// ------------------------------------------------------------ even-odd layout

size_t wd_gauge_eo_bytes(const int32_t dims[4], int32_t prec, int32_t compress12) {
  long V = 0;
  if (check_dims(dims, &V) != WD_OK || check_even_dims(dims) != WD_OK) return 0;
  if (gauge_site_bytes(prec, compress12 ? 1 : 0) == 0) return 0;
  return 2 * eo_gauge_half_bytes(V / 2, prec, compress12 ? 1 : 0);
}

size_t wd_spinor_eo_bytes(const int32_t dims[4], int32_t prec, int32_t nrhs) {
  long V = 0;
  if (check_dims(dims, &V) != WD_OK || check_even_dims(dims) != WD_OK || nrhs < 0) return 0;
  return static_cast<size_t>(packed_sites(V / 2)) * static_cast<size_t>(nrhs) * spinor_site_bytes(prec);
}

int wd_gauge_import_eo(const int32_t dims[4], const void* U_canon_dev, int32_t prec, int32_t compress12,
                       void* dst_dev, size_t dst_bytes, hipStream_t stream, wd_gauge** out) {
  try {
    clear_error();
    if (out == nullptr) return set_error(WD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    long V = 0;
    int rc = check_dims(dims, &V);
    if (rc != WD_OK) return rc;
    if ((rc = check_even_dims(dims)) != WD_OK) return rc;
    if ((rc = check_prec(prec)) != WD_OK) return rc;
    const int c12 = compress12 ? 1 : 0;
    const size_t need = 2 * eo_gauge_half_bytes(V / 2, prec, c12);
    if (dst_bytes < need) return set_error(WD_ERR_INVALID_ARG, "dst_bytes %zu < %zu needed", dst_bytes, need);
    const size_t canon_bytes = static_cast<size_t>(V) * 36 * 16;
    if ((rc = check_device_range(U_canon_dev, canon_bytes, "U_canon_dev")) != WD_OK) return rc;
    if ((rc = check_device_range(dst_dev, need, "dst_dev")) != WD_OK) return rc;
    if (overlaps(U_canon_dev, canon_bytes, dst_dev, need))
      return set_error(WD_ERR_INVALID_ARG, "U_canon_dev and dst_dev overlap");
    wd_gauge* g = new (std::nothrow) wd_gauge;
    if (g == nullptr) return set_error(WD_ERR_NOMEM, "host allocation of the handle failed");
    g->magic = kGaugeMagic;
    for (int i = 0; i < 4; ++i) g->dims[i] = dims[i];
    g->V = V;
    g->prec = prec;
    g->c12 = c12;
    g->eo = 1;
    (void)hipGetDevice(&g->device);
    g->links = dst_dev;
    g->link_bytes = need;
    rc = launch_status(launch_pack_gauge_eo(U_canon_dev, dst_dev, make_eo_geo(dims), prec, c12, stream),
                       "pack_gauge_eo");
    if (rc != WD_OK) {
      g->magic = 0;
      delete g;
      return rc;
    }
    *out = g;
    return WD_OK;
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in wd_gauge_import_eo");
  }
}

static int spinor_transfer_eo(const wd_gauge* g, const void* src, int32_t prec, int32_t nrhs, int32_t parity,
                              void* dst, hipStream_t stream, bool import) {
  int rc = check_gauge(g);
  if (rc != WD_OK) return rc;
  if ((rc = check_even_dims(g->dims)) != WD_OK) return rc;
  if ((rc = check_prec(prec)) != WD_OK) return rc;
  if (prec != g->prec)
    return set_error(WD_ERR_INVALID_ARG, "spinor precision %d differs from the gauge field's %d", prec,
                     g->prec);
  if (parity != 0 && parity != 1) return set_error(WD_ERR_INVALID_ARG, "parity is %d (0 even, 1 odd)", parity);
  if (nrhs < 0) return set_error(WD_ERR_INVALID_ARG, "nrhs is %d", nrhs);
  if (nrhs == 0) return WD_OK;
  const size_t canon = static_cast<size_t>(g->V) * nrhs * 12 * 16;
  const size_t packed = static_cast<size_t>(packed_sites(g->V / 2)) * nrhs * spinor_site_bytes(prec);
  const size_t nsrc = import ? canon : packed;
  const size_t ndst = import ? packed : canon;
  if ((rc = check_device_range(src, nsrc, import ? "canon_dev" : "src_dev")) != WD_OK) return rc;
  if ((rc = check_device_range(dst, ndst, import ? "dst_dev" : "canon_dev")) != WD_OK) return rc;
  if (overlaps(src, nsrc, dst, ndst)) return set_error(WD_ERR_INVALID_ARG, "buffers overlap");
  return launch_status(launch_spinor_eo(src, dst, make_eo_geo(g->dims), prec, parity, nrhs, import, stream),
                       import ? "pack_spinor_eo" : "unpack_spinor_eo");
}

int wd_spinor_import_eo(const wd_gauge* g, const void* canon_dev, int32_t prec, int32_t nrhs, int32_t parity,
                        void* dst_dev, hipStream_t stream) {
  try {
    clear_error();
    return spinor_transfer_eo(g, canon_dev, prec, nrhs, parity, dst_dev, stream, true);
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in wd_spinor_import_eo");
  }
}

int wd_spinor_export_eo(const wd_gauge* g, const void* src_dev, int32_t prec, int32_t nrhs, int32_t parity,
                        void* canon_dev, hipStream_t stream) {
  try {
    clear_error();
    return spinor_transfer_eo(g, src_dev, prec, nrhs, parity, canon_dev, stream, false);
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in wd_spinor_export_eo");
  }
}

int dslash_apply_eo(const wd_gauge* g, const double* masses_host, int32_t nrhs, const void* in_dev,
                    void* out_dev, void* tmp_dev, int32_t prec, int32_t flags, hipStream_t stream) {
  try {
    clear_error();
    int rc = check_gauge(g);
    if (rc != WD_OK) return rc;
    if ((rc = check_layout(g, 1, "dslash_apply_eo")) != WD_OK) return rc;
    if ((rc = check_prec(prec)) != WD_OK) return rc;
    if (prec != g->prec)
      return set_error(WD_ERR_INVALID_ARG, "spinor precision %d differs from the gauge field's %d", prec,
                       g->prec);
    if (flags & ~WD_FLAG_GAMMA5) return set_error(WD_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (nrhs < 0) return set_error(WD_ERR_INVALID_ARG, "nrhs is %d", nrhs);
    if (nrhs > kMaxMultiRhs) return set_error(WD_ERR_UNSUPPORTED, "nrhs %d exceeds %d per launch", nrhs, kMaxMultiRhs);
    if (nrhs == 0) return WD_OK;
    if (masses_host == nullptr) return set_error(WD_ERR_INVALID_ARG, "masses_host is NULL");
    for (int k = 0; k < nrhs; ++k) {
      if (!std::isfinite(masses_host[k])) return set_error(WD_ERR_INVALID_ARG, "mass %d is not finite", k);
      if (masses_host[k] == -4.0)
        return set_error(WD_ERR_INVALID_ARG, "mass %d is -4: the Schur complement divides by 4 + m", k);
    }
    const size_t n = static_cast<size_t>(packed_sites(g->V / 2)) * nrhs * spinor_site_bytes(prec);
    if ((rc = check_device_range(in_dev, n, "in_dev")) != WD_OK) return rc;
    if ((rc = check_device_range(out_dev, n, "out_dev")) != WD_OK) return rc;
    if ((rc = check_device_range(tmp_dev, n, "tmp_dev")) != WD_OK) return rc;
    if (overlaps(in_dev, n, out_dev, n) || overlaps(in_dev, n, tmp_dev, n) || overlaps(out_dev, n, tmp_dev, n))
      return set_error(WD_ERR_INVALID_ARG, "in_dev, out_dev and tmp_dev must not overlap");
    RhsSet set{};
    set.n = nrhs;
    for (int k = 0; k < nrhs; ++k) set.idx[k] = k;
    const double* m = masses_host;
    // tmp = -H_eo in / 2; out = [gamma5] ((4+m) in + H_oe tmp / (2(4+m)))
    double d[kMaxRhs], c[kMaxRhs];
    for (int k = 0; k < nrhs; ++k) {
      d[k] = 0.0;
      c[k] = -0.5;
    }
    rc = launch_status(launch_eo_hop(g, 0, in_dev, nullptr, tmp_dev, set, d, c, 0, stream), "eo hop");
    if (rc != WD_OK) return rc;
    for (int k = 0; k < nrhs; ++k) {
      d[k] = 4.0 + m[k];
      c[k] = 1.0 / (2.0 * (4.0 + m[k]));
    }
    return launch_status(launch_eo_hop(g, 1, tmp_dev, in_dev, out_dev, set, d, c,
                                       (flags & WD_FLAG_GAMMA5) ? 1 : 0, stream),
                         "eo hop");
  } catch (...) {
    return set_error(WD_ERR_INTERNAL, "unexpected exception in dslash_apply_eo");
  }
}

}  // extern "C"
