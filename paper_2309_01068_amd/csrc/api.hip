// C ABI entry points: context life cycle, interface installation, apply, operator.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <new>
#include <vector>

#include "common.h"

namespace kfbi {

static std::mutex g_attr_mu;
static std::vector<int> g_attr_done;  // devices set up: kernel LDS attributes, static workspace

size_t dyn_lds_capacity(const void* kernel) {
  int dev = 0, lim = 0;
  hipFuncAttributes a{};
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      hipFuncGetAttributes(&a, kernel) != hipSuccess)
    return 0;
  return static_cast<size_t>(lim) > a.sharedSizeBytes ? static_cast<size_t>(lim) - a.sharedSizeBytes
                                                      : 0;
}

int allow_full_dyn_lds(const void* kernel) {
  const size_t cap = dyn_lds_capacity(kernel);
  if (cap == 0) {
    set_error("cannot query the LDS attributes of a kernel");
    return KFBI_E_HIP;
  }
  KFBI_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(cap)));
  return KFBI_OK;
}

int kernel_attributes() {
  int dev = 0;
  KFBI_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_attr_mu);
  for (int d : g_attr_done)
    if (d == dev) return KFBI_OK;
  KFBI_TRY(apply_kernel_attrs());
  KFBI_TRY(gmres_kernel_attrs());
  KFBI_TRY(thetal_kernel_attrs());
  KFBI_TRY(static_scratch_setup());
  g_attr_done.push_back(dev);
  return KFBI_OK;
}

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int DBuf::ensure(size_t need) {
  if (need <= bytes) return KFBI_OK;
  if (p) {
    (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  if (need == 0) return KFBI_OK;
  // a quarter of headroom: sizes that follow a slowly growing interface (crossings, arms,
  // row parts) then reallocate rarely; hipFree synchronises the device
  const size_t want = need + need / 4 + 256;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    set_error("hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    return KFBI_E_NOMEM;
  }
  bytes = want;
  return KFBI_OK;
}

void DBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

__global__ void k_sintab(int N, double* __restrict__ s64, float* __restrict__ s32) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= 2 * N) return;
  const double v = sinpi(static_cast<double>(m) / N);
  s64[m] = v;
  s32[m] = static_cast<float>(v);
}

static int check_ctx(const kfbi_ctx* c, bool need_iface) {
  if (!c) {
    set_error("null context");
    return KFBI_E_INVALID;
  }
  if (need_iface && !c->have_interface) {
    set_error("no interface installed (call kfbi_set_interface first)");
    return KFBI_E_STATE;
  }
  return KFBI_OK;
}

// Every device workspace of a context.
template <class Ctx, class F>
static void for_each_buffer(Ctx* c, F&& f) {
  using B = std::remove_reference_t<decltype((c->X))>;
  B* bufs[] = {&c->vraw, &c->X,      &c->geo,    &c->dvec,   &c->cnt,     &c->cross,  &c->hid,
                  &c->vid,    &c->lab,    &c->armcnt, &c->rowsum,  &c->armrow, &c->armpk,
                  &c->armc,   &c->armk,   &c->armsc,  &c->chpos,
                  &c->colc,   &c->lanef,  &c->bandc,  &c->cnode,  &c->ccount,
                  &c->mkloc,  &c->tmat,   &c->pdesc,  &c->rowpart, &c->ckoff, &c->cklist, &c->ckcoef, &c->ckmk, &c->mqz,
                  &c->armcoef, &c->intptr, &c->need,    &c->nodeidx, &c->nodei,
                  &c->rowptr, &c->rows,   &c->mknode, &c->ext,     &c->gstat,  &c->mq,
                  &c->armr,   &c->qpart,  &c->ring,   &c->sinT,    &c->sinT32, &c->gband,
                  &c->nodeval, &c->tmpM,  &c->gV,     &c->gH,      &c->gsc,    &c->gpart,
                  &c->gcnt,   &c->gw,     &c->gx,     &c->gr,      &c->gd};
  for (auto* b : bufs) f(*b);
}

static size_t workspace_bytes(const kfbi_ctx* c) {
  size_t t = 0;
  for_each_buffer(c, [&](const DBuf& b) { t += b.bytes; });
  return t;
}

static void release_all(kfbi_ctx* c) {
  for_each_buffer(c, [](DBuf& b) { b.release(); });
  for (int i = 0; i < kfbi_ctx::kProfPool; ++i)
    if (c->prof_ev[i]) (void)hipEventDestroy(c->prof_ev[i]);
  for (int i = 0; i < kfbi_ctx::kGmresRing; ++i)
    if (c->gev[i]) (void)hipEventDestroy(c->gev[i]);
  if (c->hstat) (void)hipHostFree(c->hstat);
  c->hstat = c->dstat = nullptr;
}

}  // namespace kfbi

using namespace kfbi;

extern "C" {

const char* kfbi_last_error(void) { return kfbi::g_err; }

int kfbi_create(const kfbi_grid* g, kfbi_ctx** out) {
  if (!g || !out) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  *out = nullptr;
  const int N = g->N;
  if (N < 64 || N > 2048 || (N & (N - 1)) != 0) {
    set_error("N must be a power of two in [64, 2048] (got %d)", N);
    return KFBI_E_INVALID;
  }
  if (!(g->side > 0.0) || !(g->c2 >= 0.0) || !std::isfinite(g->x0) || !std::isfinite(g->y0)) {
    set_error("invalid box or c2");
    return KFBI_E_INVALID;
  }
  if (g->box_bc < KFBI_BOX_ZERO || g->box_bc > KFBI_BOX_NEUMANN) {
    set_error("invalid box_bc %d", g->box_bc);
    return KFBI_E_INVALID;
  }
  if (g->box_bc == KFBI_BOX_FREESPACE && g->c2 != 0.0) {
    set_error("free-space box data is defined for the Laplacian (c2 == 0) only");
    return KFBI_E_INVALID;
  }
  if (g->box_bc == KFBI_BOX_NEUMANN && !(g->c2 > 0.0)) {
    set_error("the zero-normal-derivative box needs c2 > 0");
    return KFBI_E_INVALID;
  }
  if (g->max_markers < 16 || g->max_markers > 4096) {
    set_error("max_markers must be in [16, 4096]");
    return KFBI_E_INVALID;
  }
  if (g->max_batch < 0 || g->max_batch > 64) {
    set_error("max_batch must be in [0, 64] (got %d)", g->max_batch);
    return KFBI_E_INVALID;
  }
  kfbi_ctx* c = new (std::nothrow) kfbi_ctx();
  if (!c) {
    set_error("out of host memory");
    return KFBI_E_NOMEM;
  }
  c->x0 = g->x0;
  c->y0 = g->y0;
  c->side = g->side;
  c->N = N;
  c->h = g->side / N;
  c->c2 = g->c2;
  c->box_bc = g->box_bc;
  c->max_markers = g->max_markers;
  c->max_batch = g->max_batch > 0 ? g->max_batch : 1;
  c->stream = static_cast<hipStream_t>(g->stream);
  int st = KFBI_OK;
  auto fail = [&](int code) {
    release_all(c);
    delete c;
    return code;
  };
  if (hipGetDevice(&c->device) != hipSuccess) {
    set_error("hipGetDevice failed");
    return fail(KFBI_E_HIP);
  }
  if ((st = kernel_attributes()) != KFBI_OK) return fail(st);
  const size_t n1sq = static_cast<size_t>(N + 1) * (N + 1);
  const size_t n = N - 1;
  const int Mx = g->max_markers;
  const size_t Bx = c->max_batch;
  if ((st = c->gstat.ensure(sizeof(GeoStatus))) ||
      (st = c->hid.ensure(sizeof(int) * n1sq)) || (st = c->vid.ensure(sizeof(int) * n1sq)) ||
      (st = c->vraw.ensure(sizeof(int) * n1sq)) ||
      (st = c->lab.ensure(n1sq)) || (st = c->need.ensure(sizeof(int) * n1sq)) ||
      (st = c->nodeidx.ensure(sizeof(int) * n1sq)) ||
      (st = c->rowsum.ensure(sizeof(int) * (2 * (N + 1) + 2))) ||
      (st = c->armrow.ensure(sizeof(int) * (N + 2))) ||
      (st = c->rows.ensure(sizeof(int) * (N + 2))) ||
      (st = c->rowptr.ensure(sizeof(int) * (N + 2))) ||
      (st = c->rowpart.ensure(sizeof(int) * (N + 2))) ||
      (st = c->nodei.ensure(sizeof(int) * 6 * Mx)) ||
      (st = c->nodeval.ensure(sizeof(double) * 6 * Mx)) ||
      (st = c->mq.ensure(sizeof(double) * 5 * Mx * Bx)) ||
      (st = c->qpart.ensure(sizeof(double) * (Mx + 64) * Bx)) ||
      (st = c->ring.ensure(sizeof(double) * 8 * (N + 1) * Bx)) ||
      (st = c->sinT.ensure(sizeof(double) * 2 * N)) ||
      (st = c->sinT32.ensure(sizeof(float) * 2 * N)) ||
      // band rows of G: the sine layout needs n N values, the cosine layout 4 ceil((N+1)/4)
      // values per row for up to N+1 rows
      (st = c->gband.ensure(sizeof(double) * (N + 4) * (N + 1) * Bx)) ||
      (st = c->mqz.ensure(sizeof(double) * 5 * Mx)) ||
      (st = c->tmpM.ensure(sizeof(double) * (Bx > 4 ? Bx : 4) * Mx)) ||
      (st = gmres_alloc(c)))
    return fail(st);
  if (hipHostMalloc(&c->hstat, 4096, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer(&c->dstat, c->hstat, 0) != hipSuccess) {
    c->hstat = c->dstat = nullptr;
    set_error("hipHostMalloc (coherent status ring) failed");
    return fail(KFBI_E_NOMEM);
  }
  if (hipMemsetAsync(c->mqz.p, 0, c->mqz.bytes, c->stream) != hipSuccess ||
      hipMemsetAsync(c->tmpM.p, 0, c->tmpM.bytes, c->stream) != hipSuccess) {
    set_error("hipMemsetAsync failed");
    return fail(KFBI_E_HIP);
  }
  hipLaunchKernelGGL(k_sintab, dim3((2 * N + 255) / 256), dim3(256), 0, c->stream, N,
                     c->sinT.as<double>(), c->sinT32.as<float>());
  if ((st = colconst_setup(c)) != KFBI_OK) return fail(st);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
    set_error("sine table kernel failed");
    return fail(KFBI_E_HIP);
  }
  *out = c;
  return KFBI_OK;
}

int kfbi_destroy(kfbi_ctx* c) {
  if (!c) return KFBI_OK;
  (void)hipStreamSynchronize(c->stream);
  release_all(c);
  delete c;
  return KFBI_OK;
}

int kfbi_set_interface(kfbi_ctx* c, int M, const double* xy) {
  KFBI_TRY(check_ctx(c, false));
  if (!xy || M < 16 || M > c->max_markers || (M & 1)) {
    set_error("M must be even and in [16, max_markers] with a non-null xy (M=%d)", M);
    return KFBI_E_INVALID;
  }
  c->have_interface = 0;
  c->last_layer = -1;
  // markers per derivative / interpolation chunk; at most 16 (M <= 4096), so a chunk has
  // at most 96 stencil nodes, which the interpolation kernel keeps two per lane
  c->mk_chunk = M >= 512 ? M / 256 : 1;
  c->n_mk_blocks = (M + c->mk_chunk - 1) / c->mk_chunk;
  const int st = geometry_setup(c, M, xy);
  if (st != KFBI_OK) return st;
  // the column solve keeps the four-mode slab of every row part of its column group in
  // LDS: 32 bytes per part (FP64)
  const size_t need = 32 * static_cast<size_t>(c->st.n_parts > 0 ? c->st.n_parts : 1);
  const size_t cap = colsolve_lds_capacity(c);
  if (need > cap) {
    set_error("interface needs %d row parts; the column solve holds at most %zu in LDS",
              c->st.n_parts, cap / 32);
    return KFBI_E_GEOMETRY;
  }
  c->have_interface = 1;
  return KFBI_OK;
}

// Densities per launch of a batched apply: as many as keep the launch's row-transform
// output (P part rows) and band (the rows the node kernel reads), FP64, within the
// 256 MB last-level cache; at least 1, at most max_batch.
static int sub_batch(const kfbi_ctx* c) {
  constexpr double kSubBatchBytes = 256.0 * 1024 * 1024;
  const double per = 8.0 * 4 * ((c->N + 4) / 4) *
                     (c->st.n_parts + (c->st.row_hi - c->st.row_lo + 1));
  const int sb = per > 0.0 ? static_cast<int>(kSubBatchBytes / per) : c->max_batch;
  return sb < 1 ? 1 : (sb > c->max_batch ? c->max_batch : sb);
}

int kfbi_get_info(const kfbi_ctx* c, kfbi_info* info) {
  KFBI_TRY(check_ctx(c, true));
  if (!info) {
    set_error("null info");
    return KFBI_E_INVALID;
  }
  info->M = c->M;
  info->n_cross_h = c->st.n_cross_h;
  info->n_cross_v = c->st.n_cross_v;
  info->n_arms = c->st.n_arms;
  info->n_nodes = c->st.n_nodes;
  info->n_rows = c->st.n_rows;
  info->row_lo = c->st.row_lo;
  info->row_hi = c->st.row_hi;
  info->n_parts = c->st.n_parts;
  info->sub_batch = sub_batch(c);
  info->workspace_bytes = static_cast<long long>(workspace_bytes(c));
  return KFBI_OK;
}

int kfbi_apply(kfbi_ctx* c, int layer, int precision, const double* dens, const double* ring,
               const kfbi_out* out) {
  KFBI_TRY(check_ctx(c, true));
  if (!dens || !out) {
    set_error("null density or output struct");
    return KFBI_E_INVALID;
  }
  if (layer != KFBI_SINGLE && layer != KFBI_DOUBLE) {
    set_error("invalid layer %d", layer);
    return KFBI_E_INVALID;
  }
  if (precision != KFBI_FP64 && precision != KFBI_FP32) {
    set_error("invalid precision %d", precision);
    return KFBI_E_INVALID;
  }
  if ((c->box_bc == KFBI_BOX_USER) != (ring != nullptr)) {
    set_error("ring values must be given exactly when box_bc == KFBI_BOX_USER");
    return KFBI_E_INVALID;
  }
  return apply_impl(c, layer, precision, dens, ring, out, nullptr, nullptr, nullptr);
}

int kfbi_apply_batch(kfbi_ctx* c, int layer, int precision, int B, const double* dens,
                     const double* ring, const kfbi_out* out) {
  KFBI_TRY(check_ctx(c, true));
  if (!dens || !out) {
    set_error("null density or output struct");
    return KFBI_E_INVALID;
  }
  if (B < 1 || B > c->max_batch) {
    set_error("batch %d outside [1, max_batch = %d]", B, c->max_batch);
    return KFBI_E_INVALID;
  }
  if (out->grid) {
    set_error("the grid output is not available for a batch");
    return KFBI_E_INVALID;
  }
  if (layer != KFBI_SINGLE && layer != KFBI_DOUBLE) {
    set_error("invalid layer %d", layer);
    return KFBI_E_INVALID;
  }
  if (precision != KFBI_FP64 && precision != KFBI_FP32) {
    set_error("invalid precision %d", precision);
    return KFBI_E_INVALID;
  }
  if ((c->box_bc == KFBI_BOX_USER) != (ring != nullptr)) {
    set_error("ring values must be given exactly when box_bc == KFBI_BOX_USER");
    return KFBI_E_INVALID;
  }
  // consecutive launches of at most sub_batch densities, sizes as equal as possible
  // (slices of the same arrays)
  const int SB = sub_batch(c);
  const int nl = (B + SB - 1) / SB;
  const size_t M = static_cast<size_t>(c->M), R = 4 * static_cast<size_t>(c->N + 1);
  for (int l = 0, b0 = 0; l < nl; ++l) {
    const int nb = B / nl + (l < B % nl ? 1 : 0);
    auto at = [&](double* p) { return p ? p + b0 * M : nullptr; };
    const kfbi_out o{at(out->v_plus), at(out->v_minus), at(out->dn_plus), at(out->dn_minus),
                     nullptr};
    KFBI_TRY(apply_impl(c, layer, precision, dens + b0 * M, ring ? ring + b0 * R : nullptr, &o,
                        nullptr, nullptr, nullptr, nb));
    b0 += nb;
  }
  return KFBI_OK;
}

int kfbi_operator(kfbi_ctx* c, const kfbi_bie* op, int precision, const double* x, double* y) {
  KFBI_TRY(check_ctx(c, true));
  if (!op || !x || !y) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  if ((op->layer != KFBI_SINGLE && op->layer != KFBI_DOUBLE) || op->side < KFBI_PLUS ||
      op->side > KFBI_AVG || (precision != KFBI_FP64 && precision != KFBI_FP32)) {
    set_error("invalid operator description");
    return KFBI_E_INVALID;
  }
  if (c->box_bc == KFBI_BOX_USER) {
    set_error("the boundary operator needs box data defined by the density (ZERO or FREESPACE)");
    return KFBI_E_INVALID;
  }
  return apply_impl(c, op->layer, precision, x, nullptr, nullptr, op, x, y);
}

int kfbi_profile(kfbi_ctx* c, int on) {
  KFBI_TRY(check_ctx(c, false));
  if (on) {
    for (int i = 0; i < kfbi_ctx::kProfPool; ++i)
      if (!c->prof_ev[i]) KFBI_HIP(hipEventCreate(&c->prof_ev[i]));
    KFBI_HIP(hipStreamSynchronize(c->stream));
    c->prof_used = 0;
    c->prof_count = 0;
    for (double& v : c->prof_ms) v = 0.0;
    c->prof_on = 1;
  } else {
    if (c->prof_on) KFBI_TRY(prof_flush(c));
    c->prof_on = 0;
  }
  return KFBI_OK;
}

int kfbi_profile_read(kfbi_ctx* c, double* ms_total, long* napplies) {
  KFBI_TRY(check_ctx(c, false));
  if (!ms_total || !napplies) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  if (c->prof_on) KFBI_TRY(prof_flush(c));
  for (int q = 0; q < 4; ++q) ms_total[q] = c->prof_ms[q];
  *napplies = c->prof_count;
  return KFBI_OK;
}

}  // extern "C"

int kfbi_profile_kernel(kfbi_ctx* c, int stage, int reps, double* us_avg) {
  KFBI_TRY(check_ctx(c, true));
  if (!us_avg) {
    set_error("null argument");
    return KFBI_E_INVALID;
  }
  return kfbi::replay_stage(c, stage, reps, us_avg);
}
