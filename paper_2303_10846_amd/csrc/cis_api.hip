// Host side of the cis library: mesh/DVS preprocessing, validation, device
// state and the C ABI declared in include/cis.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/cis.h"
#include "cis_adjoint.h"
#include "cis_internal.h"

using namespace cis;

// Device scratch of cis_iterate_noalloc, one copy per GPU, held until the process ends: the flags (4 int32 in
// the first 256 bytes), the kResidualParts x 6 residual partial sums, and the residual history of up to
// kNoAllocMaxIter iterations.  Host code never uses the name `scratch` as an address: it takes the device
// address from hipGetSymbolAddress once per device (scratch_of_device) and passes that.
static constexpr int32_t kNoAllocMaxIter = 4096;
static constexpr size_t kScratchFlagDoubles = 32;
static constexpr size_t kScratchPartDoubles = 6 * (size_t)kResidualParts;
static constexpr size_t kScratchDoubles = kScratchFlagDoubles + kScratchPartDoubles + 6 * (size_t)kNoAllocMaxIter;
static constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

thread_local std::string g_err;

cis_status fail(cis_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(CIS_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// A face identified by its node ids, sorted (a triangle has d = -1)
struct FaceId {
  int32_t a, b, c, d;
  bool operator==(const FaceId& o) const { return a == o.a && b == o.b && c == o.c && d == o.d; }
};
struct FaceIdHash {
  size_t operator()(const FaceId& k) const {
    uint64_t h = (uint64_t)(uint32_t)k.a * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)(uint32_t)k.b + 0x7F4A7C159E3779B9ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)(uint32_t)k.c + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
    h ^= (uint64_t)(uint32_t)k.d + 0xD6E8FEB86659FD93ull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};
FaceId face_id(const int32_t* v, int n) {
  int32_t t[4] = {v[0], v[1], v[2], n == 4 ? v[3] : -1};
  std::sort(t, t + n);
  return {t[0], t[1], t[2], t[3]};
}

// Local faces of the cell kinds, by node count (4 tetrahedron: the face opposite local vertex a; 5 pyramid:
// base quad 0-3 and apex 4; 6 prism: triangles 0-2 and 3-5; 8 hexahedron: quads 0-3 and 4-7), quads cyclic.
// Slot a of a cell is its a-th local face.
struct CellShape {
  int faces;
  int n[6];
  int v[6][4];
};
const CellShape* cell_shape(int kind) {
  static const CellShape shapes[4] = {
      {4, {3, 3, 3, 3}, {{1, 2, 3}, {2, 3, 0}, {3, 0, 1}, {0, 1, 2}}},
      {5, {4, 3, 3, 3, 3}, {{0, 1, 2, 3}, {0, 1, 4}, {1, 2, 4}, {2, 3, 4}, {3, 0, 4}}},
      {5, {3, 3, 4, 4, 4}, {{0, 1, 2}, {3, 4, 5}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}}},
      {6, {4, 4, 4, 4, 4, 4}, {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}}}};
  switch (kind) {
    case 4: return &shapes[0];
    case 5: return &shapes[1];
    case 6: return &shapes[2];
    case 8: return &shapes[3];
  }
  return nullptr;
}

inline void cross(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Vector area S and centroid c of a polygon face (3 or 4 nodes, cyclic).  Fanned about the node average m: S is
// the sum of the fan triangles' vector areas (for a quad, half the cross product of its diagonals: a closed cell
// has sum S = 0 exactly), and c the mean of their centroids weighted by their areas along S.
void polygon_face(const double* const* p, int n, double* S, double* c) {
  if (n == 3) {
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = p[1][d] - p[0][d];
      e2[d] = p[2][d] - p[0][d];
      c[d] = (p[0][d] + p[1][d] + p[2][d]) / 3.0;
    }
    cross(e1, e2, S);
    for (int d = 0; d < 3; ++d) S[d] *= 0.5;
    return;
  }
  double m[3], tS[4][3];
  for (int d = 0; d < 3; ++d) m[d] = 0.25 * (p[0][d] + p[1][d] + p[2][d] + p[3][d]);
  for (int d = 0; d < 3; ++d) S[d] = 0.0;
  for (int t = 0; t < 4; ++t) {
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = p[(t + 1) % 4][d] - p[t][d];
      e2[d] = m[d] - p[t][d];
    }
    cross(e1, e2, tS[t]);
    for (int d = 0; d < 3; ++d) {
      tS[t][d] *= 0.5;
      S[d] += tS[t][d];
    }
  }
  const double SS = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
  double wsum = 0.0;
  for (int d = 0; d < 3; ++d) c[d] = 0.0;
  for (int t = 0; t < 4; ++t) {
    const double wt = (tS[t][0] * S[0] + tS[t][1] * S[1] + tS[t][2] * S[2]) / SS;  // area fraction along S
    wsum += wt;
    for (int d = 0; d < 3; ++d) c[d] += wt * (p[t][d] + p[(t + 1) % 4][d] + m[d]) / 3.0;
  }
  for (int d = 0; d < 3; ++d) c[d] /= wsum;
}

template <class T> cis_status dmalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  HIP_TRY(hipMalloc((void**)p, n * sizeof(T)));
  return CIS_OK;
}

template <class T> cis_status upload(T** p, const std::vector<T>& v, hipStream_t st) {
  cis_status s = dmalloc(p, v.size());
  if (s != CIS_OK) return s;
  HIP_TRY(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return CIS_OK;
}

__global__ void k_zero_i32(int32_t* p, int n) {
  int i = threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

struct cis_mesh {
  int64_t nc = 0, nf = 0, n_int = 0, n_b = 0, n_colors = 0;
  int mf = 4;  // face slots per cell: 4 when every cell is a tetrahedron, else kMaxFaces
  std::vector<int64_t> color_off;
  std::vector<int32_t> spatial;  // cells in Morton order of their centroids (traversal order off the sweeps)
  std::vector<int32_t> cell_nb, cell_face, face_cell, face_tag;
  std::vector<double> V, h, xc, xf, fA, fn;  // cells: V, h, centroid; faces: centroid, area, unit normal
};

struct cis_dvs {
  int64_t n = 0;
  std::vector<double> u, w;
  double umax = 0.0;
};

struct cis_state {
  const cis_mesh* mesh = nullptr;
  const cis_dvs* dvs = nullptr;
  cis_gas gas{};
  cis_numerics num{};
  std::vector<cis_bc> bcs;
  int32_t precision = CIS_FP64;
  hipStream_t stream = nullptr;
  int device = 0;  // the HIP device current at cis_state_create
  Dev dev{};
  Bufs buf{};
  Work work{};
  // library-owned device arrays
  int32_t *d_cell_nb = nullptr, *d_cell_face = nullptr, *d_face_cell = nullptr, *d_face_bc = nullptr,
          *d_spatial = nullptr;
  float* d_cell_geo_f = nullptr;
  double *d_cell_geo = nullptr, *d_face_geo = nullptr, *d_dvs = nullptr, *d_bc = nullptr;
  float* d_dvs_f = nullptr;
  int64_t res_cap = 0;
  bool profile = false;
  double prof_ms[6] = {0, 0, 0, 0, 0, 0};
  int64_t prof_launch[6] = {0, 0, 0, 0, 0, 0};
  std::vector<void*> owned;
  ~cis_state() {
    for (void* p : owned)
      if (p) (void)hipFree(p);
  }
};

namespace {

template <class T> cis_status own_alloc(cis_state* s, T** p, size_t n) {
  cis_status st = dmalloc(p, n);
  if (st == CIS_OK) s->owned.push_back((void*)*p);
  return st;
}
template <class T> cis_status own_upload(cis_state* s, T** p, const std::vector<T>& v) {
  cis_status st = upload(p, v, s->stream);
  if (st == CIS_OK) s->owned.push_back((void*)*p);
  return st;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

cis_status check_numerics(const cis_numerics* n) {
  if (!n) return fail(CIS_E_INVALID_ARG, "numerics is NULL");
  if (!(n->cfl > 0.0) || !(n->inv_dt >= 0.0) || !(n->cfl_imp >= 0.0) || !(n->lim_K >= 0.0) || !(n->snap >= 0.0) ||
      n->n_macro < 0 || n->n_micro < 0 || n->n_macro > 100000 || n->n_micro > 100000 || n->limiter < 0 ||
      n->limiter > 4)
    return fail(CIS_E_INVALID_ARG, "numerics out of range");
  return CIS_OK;
}

void fill_dev_numerics(cis_state* s) {
  s->dev.snap = s->num.snap;
  s->dev.lim_K = s->num.lim_K;
  s->dev.inv_dt = s->num.inv_dt;
  s->dev.cfl_imp = s->num.cfl_imp;
  s->dev.limiter = s->num.limiter;
}

template <class F> cis_status dispatch(cis_state* s, F&& f) {
  if (s->precision == CIS_FP64) return f((double*)nullptr);
  return f((float*)nullptr);
}

cis_status device_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CIS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return CIS_OK;
}

// bc slot of `tag` (the last entry with that tag, as in the face table), -1 if none
int slot_of(const cis_state* s, int32_t tag) {
  int slot = -1;
  for (size_t b = 0; b < s->bcs.size(); ++b)
    if (s->bcs[b].tag == tag) slot = (int)b;
  return slot;
}

struct AdjSlots {
  int j = -1, w = -1, f = -1;
};

cis_status adj_slots(const cis_state* s, int32_t wall_tag, int32_t ff_tag, bool need_wall, AdjSlots* out) {
  AdjSlots a;
  a.j = slot_of(s, wall_tag);
  if (need_wall && a.j < 0) return fail(CIS_E_INVALID_ARG, "no boundary condition with the objective's wall tag");
  if (a.j >= 0 && s->bcs[a.j].kind == CIS_BC_WALL) a.w = a.j;
  const int f = slot_of(s, ff_tag);
  if (f >= 0 && s->bcs[f].kind == CIS_BC_FARFIELD) a.f = f;
  *out = a;
  return CIS_OK;
}

// g = v^T dR/dx + cJ dJ/dx for flat vectors x = [G | R | W | q] (v may be NULL: zero seed)
void run_vjp(cis_state* s, const double* v, double cJ, const AdjSlots& sl, double* g) {
  const int64_t P = s->mesh->nc * s->dvs->n, nc = s->mesh->nc;
  AdjArgs a{v, v ? v + P : nullptr, v ? v + 2 * P : nullptr, v ? v + 2 * P + 6 * nc : nullptr, cJ, sl.j, sl.w, sl.f,
            g, g + P, g + 2 * P, g + 2 * P + 6 * nc, s->work.gpf};
  launch_vjp(s->dev, s->buf, a, s->stream);
}

cis_status sum_gp(cis_state* s, double* gp) {
  std::vector<double> h(3 * (size_t)s->mesh->nf);
  HIP_TRY(hipMemcpyAsync(h.data(), s->work.gpf, h.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  double a[3] = {0.0, 0.0, 0.0};
  for (size_t f = 0; f < h.size() / 3; ++f)
    for (int m = 0; m < 3; ++m) a[m] += h[3 * f + m];
  for (int m = 0; m < 3; ++m) gp[m] = a[m];
  return CIS_OK;
}

// J = sum over the boundary faces of bc slot `slot` of A sum_k w (u.n)(|u|^2/2 G_f + R_f), from the face pass
cis_status objective_from_faces(cis_state* s, int slot, double* J) {
  const cis_mesh* m = s->mesh;
  std::vector<double> fm(6 * m->nf);
  HIP_TRY(hipMemcpyAsync(fm.data(), s->work.face_mac, fm.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  const int32_t tag = slot >= 0 ? s->bcs[slot].tag : INT32_MIN;
  double acc = 0.0;
  for (int64_t f = 0; f < m->nf; ++f)
    if (m->face_cell[2 * f + 1] < 0 && m->face_tag[f] == tag) acc += fm[6 * f + 4];
  *J = acc;
  return CIS_OK;
}

cis_status dev_dots(cis_state* s, const double* V, int64_t n, int nvec, const double* w, double* part, double* hdev,
                    double* host) {
  launch_dots(V, n, nvec, w, part, hdev, s->stream);
  HIP_TRY(hipMemcpyAsync(host, hdev, nvec * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CIS_OK;
}

// Face pass on the current state, then the per-face wall loads of `tag` (Eqs. 70-72 numerators) from the face
// macro fluxes, with n from the gas into the wall; F and Q receive the integrated force and heat load.
cis_status wall_faces(cis_state* s, int32_t tag, std::vector<cis_wall_face>& out, double* F, double* Q) {
  const cis_mesh* m = s->mesh;
  cis_status st = dispatch(s, [&](auto* tp) {
    using T = std::remove_pointer_t<decltype(tp)>;
    launch_recon<T>(s->dev, s->buf, s->stream);
    launch_face<T>(s->dev, s->buf, s->work, s->stream);
    return device_check("wall loads");
  });
  if (st != CIS_OK) return st;
  std::vector<double> fm(6 * m->nf);
  HIP_TRY(hipMemcpyAsync(fm.data(), s->work.face_mac, fm.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  out.clear();
  F[0] = F[1] = F[2] = 0.0;
  *Q = 0.0;
  for (int64_t f = 0; f < m->nf; ++f) {
    if (m->face_cell[2 * f + 1] >= 0 || m->face_tag[f] != tag) continue;
    const double A = m->fA[f];
    const double* n = &m->fn[3 * f];
    const double* mac = &fm[6 * f];  // A sum_k w (u.n) (G, u G, |u|^2/2 G + R, R)
    const double mom[3] = {mac[1] / A, mac[2] / A, mac[3] / A};
    const double p = mom[0] * n[0] + mom[1] * n[1] + mom[2] * n[2];
    cis_wall_face o;
    for (int d = 0; d < 3; ++d) {
      o.x[d] = m->xf[3 * f + d];
      o.n[d] = n[d];
      o.tau[d] = mom[d] - p * n[d];
    }
    o.area = A;
    o.p = p;
    o.q = mac[4] / A;
    out.push_back(o);
    for (int d = 0; d < 3; ++d) F[d] += mac[1 + d];
    *Q += mac[4];
  }
  return CIS_OK;
}

// Steps 2-6, n_iter times, on the state's stream, with the work arrays `w`; mark(it, k) runs between the stages.
template <class Mark> cis_status enqueue_iterations(cis_state* s, const Work& w, int32_t n_iter, Mark&& mark) {
  const cis_mesh* m = s->mesh;
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s->stream, w.flag, 4);
  return dispatch(s, [&](auto* tp) {
    using T = std::remove_pointer_t<decltype(tp)>;
    for (int32_t it = 0; it < n_iter; ++it) {
      mark(it, 0);
      launch_recon<T>(s->dev, s->buf, s->stream);
      mark(it, 1);
      launch_face<T>(s->dev, s->buf, w, s->stream);
      mark(it, 2);
      launch_macro(s->dev, s->buf, w, m->color_off.data(), m->n_colors, s->num.n_macro, s->stream);
      mark(it, 3);
      launch_residual<T>(s->dev, s->buf, w, s->buf.resG, s->buf.resR, 0, s->stream);
      mark(it, 4);
      launch_micro<T>(s->dev, s->buf, w, m->color_off.data(), m->n_colors, s->num.n_micro, s->stream);
      mark(it, 5);
      launch_update<T>(s->dev, s->buf, w, it, s->stream);
      mark(it, 6);
    }
    return device_check("iterate");
  });
}

// Copy the residual history (Step 7) of the last n_iter iterations and the positivity flags back; synchronises.
cis_status finish_iterations(cis_state* s, const Work& w, int32_t n_iter, double* res_hist) {
  int32_t flag[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(flag, w.flag, sizeof(flag), hipMemcpyDeviceToHost, s->stream));
  if (res_hist)
    HIP_TRY(hipMemcpyAsync(res_hist, w.res, 6 * (size_t)n_iter * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (flag[0]) return fail(CIS_E_NONFINITE, "non-finite or non-positive state (flag " + std::to_string(flag[0]) + ")");
  return CIS_OK;
}

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, looked up on the first call for that device (with it current).
cis_status scratch_of_device(int device, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return fail(CIS_E_UNSUPPORTED, "device index beyond the scratch table");
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != device) HIP_TRY(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return fail(CIS_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return CIS_OK;
}

int64_t adjoint_doubles(const cis_state* s, int32_t restart) {
  const int64_t N = 2 * s->mesh->nc * s->dvs->n + 12 * s->mesh->nc;
  return ((int64_t)restart + 4) * N + ((int64_t)restart + 2) * (dot_partials() + 1) +
         kBlockPrecondCellDoubles * s->mesh->nc;
}

}  // namespace

extern "C" {

const char* cis_last_error(void) { return g_err.c_str(); }

cis_status cis_mesh_create(const double* xyz, int64_t n_nodes, const int32_t* tet, int64_t n_cells,
                           const int32_t* btri, const int32_t* btag, int64_t n_b, const int64_t* color_offsets,
                           int64_t n_colors, cis_mesh** out) {
  if (!out) return fail(CIS_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!xyz || !tet || n_nodes <= 0 || n_cells <= 0 || n_cells > INT32_MAX || n_b < 0 || (n_b > 0 && (!btri || !btag)))
    return fail(CIS_E_INVALID_ARG, "bad mesh arrays");
  std::vector<int32_t> cells(8 * (size_t)n_cells, -1), kinds((size_t)n_cells, 4), bface(4 * (size_t)n_b, -1);
  for (int64_t i = 0; i < n_cells; ++i)
    for (int a = 0; a < 4; ++a) cells[8 * i + a] = tet[4 * i + a];
  for (int64_t b = 0; b < n_b; ++b)
    for (int a = 0; a < 3; ++a) bface[4 * b + a] = btri[3 * b + a];
  return cis_mesh_create_cells(xyz, n_nodes, cells.data(), kinds.data(), n_cells, bface.data(), btag, n_b,
                               color_offsets, n_colors, out);
}

cis_status cis_mesh_create_cells(const double* xyz, int64_t n_nodes, const int32_t* cells, const int32_t* kinds,
                                 int64_t n_cells, const int32_t* bface, const int32_t* btag, int64_t n_b,
                                 const int64_t* color_offsets, int64_t n_colors, cis_mesh** out) {
  if (!out) return fail(CIS_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!xyz || !cells || !kinds || n_nodes <= 0 || n_cells <= 0 || n_cells > INT32_MAX || n_b < 0 ||
      (n_b > 0 && (!bface || !btag)))
    return fail(CIS_E_INVALID_ARG, "bad mesh arrays");
  if (!color_offsets || n_colors <= 0) return fail(CIS_E_INVALID_ARG, "colour offsets are required");
  if (color_offsets[0] != 0 || color_offsets[n_colors] != n_cells)
    return fail(CIS_E_INVALID_ARG, "colour offsets must run from 0 to n_cells");
  for (int64_t c = 0; c < n_colors; ++c)
    if (color_offsets[c + 1] < color_offsets[c]) return fail(CIS_E_INVALID_ARG, "colour offsets must not decrease");
  if (!finite_all(xyz, 3 * (size_t)n_nodes)) return fail(CIS_E_MESH, "non-finite node coordinate");
  int mf = 4;
  for (int64_t i = 0; i < n_cells; ++i) {
    const CellShape* sh = cell_shape(kinds[i]);
    if (!sh) return fail(CIS_E_INVALID_ARG, "cell kind must be 4, 5, 6 or 8 (nodes)");
    if (sh->faces > 4) mf = kMaxFaces;
    for (int a = 0; a < kinds[i]; ++a)
      if (cells[8 * i + a] < 0 || cells[8 * i + a] >= n_nodes) return fail(CIS_E_MESH, "cell node id out of range");
  }
  for (int64_t b = 0; b < n_b; ++b) {
    const int n = bface[4 * b + 3] < 0 ? 3 : 4;
    for (int a = 0; a < n; ++a)
      if (bface[4 * b + a] < 0 || bface[4 * b + a] >= n_nodes) return fail(CIS_E_MESH, "boundary node id out of range");
  }

  auto* m = new cis_mesh();
  m->nc = n_cells;
  m->mf = mf;
  m->n_colors = n_colors;
  m->color_off.assign(color_offsets, color_offsets + n_colors + 1);
  m->cell_face.assign((size_t)mf * n_cells, -1);
  m->cell_nb.assign((size_t)mf * n_cells, kNoFace);
  m->V.resize(n_cells);
  m->xc.resize(3 * n_cells);
  // cells: a tetrahedron directly (|det|/6, vertex mean); another kind as the tetrahedra from its node average
  // to the triangles of its faces (quads fanned about their node average)
  for (int64_t i = 0; i < n_cells; ++i) {
    const int32_t* cn = cells + 8 * i;
    if (kinds[i] == 4) {
      const double* p0 = xyz + 3 * cn[0];
      const double* p1 = xyz + 3 * cn[1];
      const double* p2 = xyz + 3 * cn[2];
      const double* p3 = xyz + 3 * cn[3];
      double a[3], b[3], c[3];
      for (int d = 0; d < 3; ++d) {
        a[d] = p1[d] - p0[d];
        b[d] = p2[d] - p0[d];
        c[d] = p3[d] - p0[d];
      }
      double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) + a[2] * (b[0] * c[1] - b[1] * c[0]);
      m->V[i] = std::fabs(det) / 6.0;
      for (int d = 0; d < 3; ++d) m->xc[3 * i + d] = 0.25 * (p0[d] + p1[d] + p2[d] + p3[d]);
    } else {
      const CellShape* sh = cell_shape(kinds[i]);
      double ctr[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < kinds[i]; ++a)
        for (int d = 0; d < 3; ++d) ctr[d] += xyz[3 * cn[a] + d];
      for (int d = 0; d < 3; ++d) ctr[d] /= kinds[i];
      double vol = 0.0, mom[3] = {0.0, 0.0, 0.0};
      bool bad = false;
      for (int a = 0; a < sh->faces && !bad; ++a) {
        const int n = sh->n[a];
        const double* p[4];
        double fm[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < n; ++q) {
          p[q] = xyz + 3 * cn[sh->v[a][q]];
          for (int d = 0; d < 3; ++d) fm[d] += p[q][d] / n;
        }
        double v6[4], cq[4][3], tot = 0.0;
        const int nt = n == 3 ? 1 : 4;
        for (int t = 0; t < nt; ++t) {
          const double* x0 = n == 3 ? p[0] : p[t];
          const double* x1 = n == 3 ? p[1] : p[(t + 1) % 4];
          const double* x2 = n == 3 ? p[2] : fm;
          double e1[3], e2[3], e3[3], cr[3];
          for (int d = 0; d < 3; ++d) {
            e1[d] = x1[d] - x0[d];
            e2[d] = x2[d] - x0[d];
            e3[d] = ctr[d] - x0[d];
            cq[t][d] = 0.25 * (x0[d] + x1[d] + x2[d] + ctr[d]);
          }
          cross(e1, e2, cr);
          v6[t] = cr[0] * e3[0] + cr[1] * e3[1] + cr[2] * e3[2];  // 6 x signed volume
          tot += v6[t];
        }
        for (int t = 0; t < nt; ++t) {
          const double v = (tot < 0.0 ? -v6[t] : v6[t]) / 6.0;
          if (!(v > 0.0)) bad = true;
          vol += v;
          for (int d = 0; d < 3; ++d) mom[d] += v * cq[t][d];
        }
      }
      if (bad) {
        delete m;
        return fail(CIS_E_MESH, "cell " + std::to_string(i) + " is folded");
      }
      m->V[i] = vol;
      for (int d = 0; d < 3; ++d) m->xc[3 * i + d] = mom[d] / vol;
    }
    if (!(m->V[i] > 0.0)) {
      delete m;
      return fail(CIS_E_MESH, "cell " + std::to_string(i) + " has zero volume");
    }
  }
  // Morton order of the centroids: kernels that read face neighbours walk the cells in this order, so that
  // neighbouring rows are read close together in time (the colour-major numbering puts every face neighbour
  // of a cell in another colour block)
  {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < n_cells; ++i)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], m->xc[3 * i + d]);
        hi[d] = std::max(hi[d], m->xc[3 * i + d]);
      }
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)n_cells);
    for (int64_t i = 0; i < n_cells; ++i) {
      uint64_t code = 0;
      for (int d = 0; d < 3; ++d) {
        const double t = hi[d] > lo[d] ? (m->xc[3 * i + d] - lo[d]) / (hi[d] - lo[d]) : 0.0;
        const uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, t * 2097152.0));
        for (int b = 0; b < 21; ++b) code |= ((q >> b) & 1ull) << (3 * b + d);
      }
      key[(size_t)i] = {code, (int32_t)i};
    }
    std::sort(key.begin(), key.end());
    m->spatial.resize((size_t)n_cells);
    for (int64_t i = 0; i < n_cells; ++i) m->spatial[(size_t)i] = key[(size_t)i].second;
  }
  // faces: slot a of a cell is its a-th local face
  std::unordered_map<FaceId, int64_t, FaceIdHash> seen;
  seen.reserve((size_t)(3 * n_cells));
  std::vector<FaceId> fkey;
  std::vector<std::array<int32_t, 4>> fcyc;  // the face's nodes in the first cell's cyclic order
  for (int64_t i = 0; i < n_cells; ++i) {
    const CellShape* sh = cell_shape(kinds[i]);
    for (int a = 0; a < sh->faces; ++a) {
      std::array<int32_t, 4> v = {-1, -1, -1, -1};
      for (int q = 0; q < sh->n[a]; ++q) v[q] = cells[8 * i + sh->v[a][q]];
      FaceId key = face_id(v.data(), sh->n[a]);
      auto it = seen.find(key);
      if (it == seen.end()) {
        int64_t f = (int64_t)fkey.size();
        seen.emplace(key, f);
        fkey.push_back(key);
        fcyc.push_back(v);
        m->face_cell.push_back((int32_t)i);
        m->face_cell.push_back(-1);
        m->cell_face[(size_t)mf * i + a] = (int32_t)f;
      } else {
        int64_t f = it->second;
        if (m->face_cell[2 * f + 1] != -1 || m->face_cell[2 * f] == (int32_t)i) {
          delete m;
          return fail(CIS_E_MESH, "non-manifold face");
        }
        m->face_cell[2 * f + 1] = (int32_t)i;
        m->cell_face[(size_t)mf * i + a] = (int32_t)f;
      }
    }
  }
  m->nf = (int64_t)fkey.size();
  m->face_tag.assign(m->nf, 0);
  std::unordered_map<FaceId, int32_t, FaceIdHash> tags;
  for (int64_t b = 0; b < n_b; ++b) tags[face_id(bface + 4 * b, bface[4 * b + 3] < 0 ? 3 : 4)] = btag[b];
  m->n_int = 0;
  m->n_b = 0;
  for (int64_t f = 0; f < m->nf; ++f) {
    if (m->face_cell[2 * f + 1] >= 0) {
      ++m->n_int;
      continue;
    }
    auto it = tags.find(fkey[f]);
    if (it == tags.end()) {
      delete m;
      return fail(CIS_E_MESH, "open face without a boundary tag");
    }
    m->face_tag[f] = it->second;
    ++m->n_b;
  }
  // face geometry; interior faces get the canonical orientation (first normal component beyond 1e-9 > 0)
  m->xf.resize(3 * m->nf);
  m->fA.resize(m->nf);
  m->fn.resize(3 * m->nf);
  for (int64_t f = 0; f < m->nf; ++f) {
    double n[3], len;
    if (fkey[f].d < 0) {
      // a triangle, from its sorted node ids
      const double* a = xyz + 3 * fkey[f].a;
      const double* b = xyz + 3 * fkey[f].b;
      const double* c = xyz + 3 * fkey[f].c;
      double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
      cross(e1, e2, n);
      len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      for (int d = 0; d < 3; ++d) m->xf[3 * f + d] = (a[d] + b[d] + c[d]) / 3.0;
    } else {
      const double* p[4];
      for (int q = 0; q < 4; ++q) p[q] = xyz + 3 * fcyc[f][q];
      double S[3];
      polygon_face(p, 4, S, &m->xf[3 * f]);
      for (int d = 0; d < 3; ++d) n[d] = 2.0 * S[d];
      len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    }
    if (!(len > 0.0)) {
      delete m;
      return fail(CIS_E_MESH, "degenerate face");
    }
    for (int d = 0; d < 3; ++d) n[d] /= len;
    m->fA[f] = 0.5 * len;
    int32_t o = m->face_cell[2 * f];
    double dot = 0.0;
    for (int d = 0; d < 3; ++d) dot += n[d] * (m->xf[3 * f + d] - m->xc[3 * o + d]);
    if (dot < 0.0)
      for (int d = 0; d < 3; ++d) n[d] = -n[d];
    if (m->face_cell[2 * f + 1] >= 0) {
      int d0 = 0;
      while (d0 < 2 && std::fabs(n[d0]) <= 1e-9) ++d0;
      if (n[d0] < 0.0) {
        for (int d = 0; d < 3; ++d) n[d] = -n[d];
        std::swap(m->face_cell[2 * f], m->face_cell[2 * f + 1]);
      }
    }
    for (int d = 0; d < 3; ++d) m->fn[3 * f + d] = n[d];
  }
  // neighbours, closure, h, colouring
  m->h.resize(n_cells);
  for (int64_t i = 0; i < n_cells; ++i) {
    double acc[3] = {0, 0, 0}, asum = 0.0;
    for (int a = 0; a < mf; ++a) {
      int64_t f = m->cell_face[(size_t)mf * i + a];
      if (f < 0) continue;
      bool own = m->face_cell[2 * f] == (int32_t)i;
      m->cell_nb[(size_t)mf * i + a] = own ? m->face_cell[2 * f + 1] : m->face_cell[2 * f];
      double sg = own ? 1.0 : -1.0;
      for (int d = 0; d < 3; ++d) acc[d] += sg * m->fA[f] * m->fn[3 * f + d];
      asum += m->fA[f];
    }
    if (std::sqrt(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]) > 1e-10 * asum) {
      delete m;
      return fail(CIS_E_MESH, "cell " + std::to_string(i) + " is not closed");
    }
    m->h[i] = 6.0 * m->V[i] / asum;
  }
  std::vector<int32_t> color(n_cells);
  for (int64_t c = 0; c < n_colors; ++c)
    for (int64_t i = color_offsets[c]; i < color_offsets[c + 1]; ++i) color[i] = (int32_t)c;
  for (int64_t f = 0; f < m->nf; ++f) {
    int32_t j = m->face_cell[2 * f + 1];
    if (j >= 0 && color[j] == color[m->face_cell[2 * f]]) {
      delete m;
      return fail(CIS_E_MESH, "two face neighbours share a colour");
    }
  }
  *out = m;
  return CIS_OK;
}

cis_status cis_mesh_info(const cis_mesh* m, cis_mesh_info_t* out) {
  if (!m || !out) return fail(CIS_E_INVALID_ARG, "NULL argument");
  out->n_cells = m->nc;
  out->n_faces = m->nf;
  out->n_interior = m->n_int;
  out->n_boundary = m->n_b;
  out->n_colors = m->n_colors;
  out->max_faces = m->mf;
  return CIS_OK;
}

void cis_mesh_destroy(cis_mesh* m) { delete m; }

cis_status cis_dvs_create(const double* u, const double* w, int64_t n, cis_dvs** out) {
  if (!out) return fail(CIS_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!u || !w || n <= 0) return fail(CIS_E_INVALID_ARG, "bad DVS arrays");
  if (!finite_all(u, 3 * (size_t)n)) return fail(CIS_E_DVS, "non-finite velocity");
  for (int64_t k = 0; k < n; ++k)
    if (!(w[k] > 0.0) || !std::isfinite(w[k])) return fail(CIS_E_DVS, "DVS weight must be positive");
  auto* d = new cis_dvs();
  d->n = n;
  d->u.assign(u, u + 3 * n);
  d->w.assign(w, w + n);
  for (int64_t k = 0; k < n; ++k)
    d->umax = std::max(d->umax, std::sqrt(u[3 * k] * u[3 * k] + u[3 * k + 1] * u[3 * k + 1] + u[3 * k + 2] * u[3 * k + 2]));
  if (!(d->umax > 0.0)) {
    delete d;
    return fail(CIS_E_DVS, "all velocities are zero");
  }
  *out = d;
  return CIS_OK;
}

void cis_dvs_destroy(cis_dvs* d) { delete d; }

cis_status cis_state_required_bytes(const cis_mesh* m, const cis_dvs* d, int32_t precision, cis_buffer_sizes* out) {
  if (!m || !d || !out) return fail(CIS_E_INVALID_ARG, "NULL argument");
  if (precision != CIS_FP64 && precision != CIS_MIXED) return fail(CIS_E_INVALID_ARG, "unknown precision");
  int64_t es = precision == CIS_FP64 ? 8 : 4;
  out->phi_bytes = m->nc * d->n * es;
  out->face_bytes = m->nf * d->n * es;
  out->cell6_bytes = m->nc * 6 * 8;
  out->code_bytes = m->nc * d->n * (m->mf == 4 ? 1 : 2);
  out->total_bytes = 6 * out->phi_bytes + 2 * out->face_bytes + 2 * out->cell6_bytes + out->code_bytes;
  return CIS_OK;
}

cis_status cis_state_create(const cis_mesh* m, const cis_dvs* dv, const cis_gas* gas, const cis_numerics* num,
                            const cis_bc* bc, int32_t n_bc, int32_t precision, const cis_device_buffers* buf,
                            void* stream, cis_state** out) {
  if (!out) return fail(CIS_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!m || !dv || !gas || !buf || (n_bc > 0 && !bc) || n_bc < 0) return fail(CIS_E_INVALID_ARG, "NULL argument");
  if (precision != CIS_FP64 && precision != CIS_MIXED) return fail(CIS_E_INVALID_ARG, "unknown precision");
  cis_status st = check_numerics(num);
  if (st != CIS_OK) return st;
  if (num->limiter >= 3) return fail(CIS_E_INVALID_ARG, "limiters 3 and 4 need stored values: cis_limiter_freeze first");
  if (!buf->G || !buf->R || !buf->dG || !buf->dR || !buf->resG || !buf->resR || !buf->faceG || !buf->faceR || !buf->W ||
      !buf->q || !buf->upwind)
    return fail(CIS_E_INVALID_ARG, "a device buffer is NULL");
  if (!(gas->R > 0) || !(gas->gamma > 1) || !(gas->Z > 0) || !(gas->mu_ref > 0) || !(gas->T_ref > 0) ||
      !(gas->C_s >= 0) || !std::isfinite(gas->C_s))
    return fail(CIS_E_INVALID_ARG, "gas constants out of range");
  if (dv->n > (int64_t)max_velocities())
    return fail(CIS_E_UNSUPPORTED, "velocity set larger than " + std::to_string(max_velocities()));
  for (int b = 0; b < n_bc; ++b) {
    if ((bc[b].kind != CIS_BC_WALL && bc[b].kind != CIS_BC_FARFIELD) || !(bc[b].T > 0.0) ||
        (bc[b].kind == CIS_BC_FARFIELD && !(bc[b].rho > 0.0)))
      return fail(CIS_E_INVALID_ARG, "bad boundary condition " + std::to_string(b));
  }
  std::vector<int32_t> face_bc(m->nf, -1);
  for (int64_t f = 0; f < m->nf; ++f) {
    if (m->face_cell[2 * f + 1] >= 0) continue;
    int slot = -1;
    for (int b = 0; b < n_bc; ++b)
      if (bc[b].tag == m->face_tag[f]) slot = b;
    if (slot < 0) return fail(CIS_E_INVALID_ARG, "no boundary condition for tag " + std::to_string(m->face_tag[f]));
    face_bc[f] = slot;
  }

  auto* s = new cis_state();
  s->mesh = m;
  s->dvs = dv;
  s->gas = *gas;
  s->num = *num;
  s->bcs.assign(bc, bc + n_bc);
  s->precision = precision;
  s->stream = (hipStream_t)stream;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(CIS_E_DEVICE, "hipGetDevice failed");
  }
  const int64_t nc = m->nc, nf = m->nf, nv = dv->n;

  // geometry that depends on the DVS: dt_i = cfl h_i / max|u|, s_f, Delta l_f, least-squares weights
  std::vector<double> dt(nc);
  for (int64_t i = 0; i < nc; ++i) dt[i] = num->cfl * m->h[i] / dv->umax;
  std::vector<double> fgeo(FGW * nf, 0.0);
  for (int64_t f = 0; f < nf; ++f) {
    int32_t i = m->face_cell[2 * f], j = m->face_cell[2 * f + 1];
    double* g = &fgeo[FGW * f];
    g[0] = m->fA[f];
    for (int d = 0; d < 3; ++d) g[1 + d] = m->fn[3 * f + d];
    double d2 = 0.0;
    if (j >= 0) {
      g[4] = std::min(dt[i], dt[j]);
      for (int d = 0; d < 3; ++d) d2 += (m->xc[3 * i + d] - m->xc[3 * j + d]) * (m->xc[3 * i + d] - m->xc[3 * j + d]);
      g[5] = std::sqrt(d2);
    } else {
      g[4] = dt[i];
      for (int d = 0; d < 3; ++d) d2 += (m->xf[3 * f + d] - m->xc[3 * i + d]) * (m->xf[3 * f + d] - m->xc[3 * i + d]);
      g[5] = 2.0 * std::sqrt(d2);
    }
  }
  const int mf = m->mf;
  const int cgw = mf == 4 ? Lay<4>::CG : Lay<kMaxFaces>::CG;
  const int cgfw = mf == 4 ? Lay<4>::CGF : Lay<kMaxFaces>::CGF;
  std::vector<double> cgeo((size_t)cgw * nc, 0.0);
  for (int64_t i = 0; i < nc; ++i) {
    double* g = &cgeo[(size_t)cgw * i];
    g[0] = m->V[i];
    g[1] = 1.0 / m->V[i];
    g[2] = m->h[i];
    for (int d = 0; d < 3; ++d) g[4 + d] = m->xc[3 * i + d];
    double M[9] = {0}, dvec[kMaxFaces][3];
    for (int a = 0; a < mf; ++a) {
      int64_t f = m->cell_face[(size_t)mf * i + a];
      int32_t nb = m->cell_nb[(size_t)mf * i + a];
      if (f < 0) continue;  // unused slot: zero geometry
      double sg = m->face_cell[2 * f] == (int32_t)i ? 1.0 : -1.0;
      double* sl = g + CG_FACE + CG_SLOT * a;
      sl[0] = sg;
      sl[1] = m->fA[f] / m->V[i];
      for (int d = 0; d < 3; ++d) {
        sl[2 + d] = sg * m->fn[3 * f + d];
        sl[5 + d] = m->xf[3 * f + d] - m->xc[3 * i + d];
        dvec[a][d] = (nb >= 0 ? m->xc[3 * nb + d] : m->xf[3 * f + d]) - m->xc[3 * i + d];
      }
      sl[8] = fgeo[FGW * f + 4];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] += dvec[a][r] * dvec[a][c];
    }
    // inverse of the least-squares normal matrix (unweighted; boundary faces enter with a zero difference)
    double c00 = M[4] * M[8] - M[5] * M[7], c01 = M[5] * M[6] - M[3] * M[8], c02 = M[3] * M[7] - M[4] * M[6];
    double det = M[0] * c00 + M[1] * c01 + M[2] * c02;
    if (!(std::fabs(det) > 0.0)) {
      delete s;
      return fail(CIS_E_MESH, "singular least-squares matrix");
    }
    double I[9] = {c00, M[2] * M[7] - M[1] * M[8], M[1] * M[5] - M[2] * M[4],
                   c01, M[0] * M[8] - M[2] * M[6], M[2] * M[3] - M[0] * M[5],
                   c02, M[1] * M[6] - M[0] * M[7], M[0] * M[4] - M[1] * M[3]};
    for (int a = 0; a < mf; ++a) {
      double* sl = g + CG_FACE + CG_SLOT * a;
      bool interior = m->cell_nb[(size_t)mf * i + a] >= 0;
      for (int r = 0; r < 3; ++r)
        sl[9 + r] = interior ? (I[3 * r] * dvec[a][0] + I[3 * r + 1] * dvec[a][1] + I[3 * r + 2] * dvec[a][2]) / det : 0.0;
    }
  }
  std::vector<float> cgeof((size_t)cgfw * nc, 0.0f);
  for (int64_t i = 0; i < nc; ++i)
    for (int a = 0; a < mf; ++a) {
      const double* sl = &cgeo[(size_t)cgw * i + CG_FACE + CG_SLOT * a];
      float* o = &cgeof[(size_t)cgfw * i + 7 * a];
      for (int q = 0; q < 3; ++q) {
        o[q] = (float)sl[5 + q];
        o[4 + q] = (float)sl[9 + q];
      }
      o[3] = (float)sl[8];
    }
  std::vector<double> dvsv(DVS_ARRAYS * nv, 0.0);
  std::vector<float> dvsf(DVS_F_ARRAYS * nv, 0.0f);
  for (int64_t k = 0; k < nv; ++k) {
    const double* u = &dv->u[3 * k];
    double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int d = 0; d < 3; ++d) {
      dvsv[d * nv + k] = u[d];
      dvsf[d * nv + k] = (float)u[d];
    }
    dvsv[3 * nv + k] = dv->w[k];
    dvsv[4 * nv + k] = std::sqrt(u2);
    dvsv[5 * nv + k] = 0.5 * u2;
  }
  std::vector<double> bct(BCW * std::max(n_bc, 1), 0.0);
  for (int b = 0; b < n_bc; ++b) {
    double* p = &bct[BCW * b];
    p[0] = bc[b].kind;
    p[1] = bc[b].rho;
    for (int d = 0; d < 3; ++d) p[2 + d] = bc[b].U[d];
    p[5] = bc[b].T;
  }
  cis_status e = CIS_OK;
  auto chk = [&](cis_status x) {
    if (e == CIS_OK) e = x;
  };
  chk(own_upload(s, &s->d_cell_nb, m->cell_nb));
  chk(own_upload(s, &s->d_spatial, m->spatial));
  chk(own_upload(s, &s->d_cell_face, m->cell_face));
  chk(own_upload(s, &s->d_face_cell, m->face_cell));
  chk(own_upload(s, &s->d_face_bc, face_bc));
  chk(own_upload(s, &s->d_cell_geo, cgeo));
  chk(own_upload(s, &s->d_cell_geo_f, cgeof));
  chk(own_upload(s, &s->d_face_geo, fgeo));
  chk(own_upload(s, &s->d_dvs, dvsv));
  chk(own_upload(s, &s->d_dvs_f, dvsf));
  chk(own_upload(s, &s->d_bc, bct));
  Work& w = s->work;
  chk(own_alloc(s, &w.face_mac, 6 * nf));
  chk(own_alloc(s, &w.cell_prim, 8 * nc));
  chk(own_alloc(s, &w.rcf, (size_t)mf * nc));
  chk(own_alloc(s, &w.G0, (size_t)6 * mf * nc));
  chk(own_alloc(s, &w.mres, 6 * nc));
  chk(own_alloc(s, &w.mD, 2 * nc));
  chk(own_alloc(s, &w.Fmac, 6 * nc));
  chk(own_alloc(s, &w.dW, 6 * nc));
  chk(own_alloc(s, &w.mbase, nc));
  chk(own_alloc(s, &w.Wt, 6 * nc));
  chk(own_alloc(s, &w.eq, ER * nc));
  chk(own_alloc(s, &w.cellres, 6 * nc));
  chk(own_alloc(s, &w.flag, 4));
  chk(own_alloc(s, &w.respart, 6 * 256));
  chk(own_alloc(s, &w.gpf, 3 * nf));
  s->res_cap = 64;
  chk(own_alloc(s, &w.res, 6 * s->res_cap));
  if (e != CIS_OK) {
    delete s;
    return e;
  }
  if (hipStreamSynchronize(s->stream) != hipSuccess) {
    delete s;
    return fail(CIS_E_DEVICE, "upload failed");
  }
  Dev& d = s->dev;
  d.nc = nc;
  d.nf = nf;
  d.nv = nv;
  d.mf = mf;
  d.cell_nb = s->d_cell_nb;
  d.spatial = s->d_spatial;
  d.cell_face = s->d_cell_face;
  d.cell_geo = s->d_cell_geo;
  d.cell_geo_f = s->d_cell_geo_f;
  d.upw = buf->upwind;
  d.face_cell = s->d_face_cell;
  d.face_bc = s->d_face_bc;
  d.face_geo = s->d_face_geo;
  d.dvs = s->d_dvs;
  d.dvs_f = s->d_dvs_f;
  d.bc = s->d_bc;
  d.gas = GasC{gas->R,      gas->gamma,  gas->Z,         gas->delta, gas->omega0,
               gas->omega1, gas->mu_ref, gas->omega_vhs, gas->T_ref, gas->C_s};
  d.umax = dv->umax;
  d.lim_frozen = nullptr;
  fill_dev_numerics(s);
  s->buf = Bufs{buf->G, buf->R, buf->dG, buf->dR, buf->resG, buf->resR, buf->faceG, buf->faceR, buf->W, buf->q};
  launch_upwind_codes(d, s->stream);
  if (hipStreamSynchronize(s->stream) != hipSuccess || hipGetLastError() != hipSuccess) {
    delete s;
    return fail(CIS_E_DEVICE, "upwind codes failed");
  }
  *out = s;
  return CIS_OK;
}

cis_status cis_state_set_numerics(cis_state* s, const cis_numerics* num) {
  if (!s) return fail(CIS_E_INVALID_ARG, "state is NULL");
  cis_status st = check_numerics(num);
  if (st != CIS_OK) return st;
  if (num->cfl != s->num.cfl) return fail(CIS_E_UNSUPPORTED, "cfl (face step s_ij) is fixed at state creation");
  if (num->limiter >= 3 && !s->dev.lim_frozen)
    return fail(CIS_E_INVALID_ARG, "limiters 3 and 4 need stored values: cis_limiter_freeze first");
  const bool recode = num->snap != s->num.snap;
  s->num = *num;
  fill_dev_numerics(s);
  if (recode) {
    launch_upwind_codes(s->dev, s->stream);
    st = device_check("upwind codes");
    if (st != CIS_OK) return st;
  }
  return CIS_OK;
}

void cis_state_destroy(cis_state* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  delete s;
}

cis_status cis_limiter_freeze(cis_state* s, void* L, int32_t compute) {
  if (!s) return fail(CIS_E_INVALID_ARG, "state is NULL");
  if (!L) {
    if (s->num.limiter >= 3) return fail(CIS_E_INVALID_ARG, "stored limiter values are in use: set limiter 0-2 first");
    s->dev.lim_frozen = nullptr;
    return CIS_OK;
  }
  if (!compute) {
    s->dev.lim_frozen = L;
    return CIS_OK;
  }
  cis_status st = dispatch(s, [&](auto* tp) {
    using T = std::remove_pointer_t<decltype(tp)>;
    launch_recon<T>(s->dev, s->buf, s->stream, L);
    return device_check("limiter freeze");
  });
  if (st != CIS_OK) return st;
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->dev.lim_frozen = L;
  return CIS_OK;
}

cis_status cis_state_init_equilibrium(cis_state* s, const double* W0, int32_t per_cell) {
  if (!s || !W0) return fail(CIS_E_INVALID_ARG, "NULL argument");
  const int64_t nc = s->mesh->nc;
  size_t n = per_cell ? 6 * (size_t)nc : 6;
  if (!finite_all(W0, n)) return fail(CIS_E_INVALID_ARG, "non-finite W0");
  for (size_t c = 0; c < n; c += 6) {
    double ke = 0.5 * (W0[c + 1] * W0[c + 1] + W0[c + 2] * W0[c + 2] + W0[c + 3] * W0[c + 3]) / W0[c];
    if (!(W0[c] > 0.0) || !(W0[c + 5] > 0.0) || !(W0[c + 4] - ke - W0[c + 5] > 0.0))
      return fail(CIS_E_INVALID_ARG, "W0 must have rho, T_tr, T_rot > 0");
  }
  double* dW0 = nullptr;
  HIP_TRY(hipMalloc((void**)&dW0, n * sizeof(double)));
  hipError_t e1 = hipMemcpyAsync(dW0, W0, n * sizeof(double), hipMemcpyHostToDevice, s->stream);
  cis_status st = CIS_OK;
  if (e1 == hipSuccess) {
    st = dispatch(s, [&](auto* tp) {
      using T = std::remove_pointer_t<decltype(tp)>;
      launch_init_eq<T>(s->dev, s->buf, dW0, per_cell ? 1 : 0, s->work.eq, s->stream);
      return device_check("init_equilibrium");
    });
  }
  hipError_t e2 = hipStreamSynchronize(s->stream);
  (void)hipFree(dW0);
  if (e1 != hipSuccess || e2 != hipSuccess) return fail(CIS_E_DEVICE, "init_equilibrium failed");
  return st;
}

cis_status cis_state_set(cis_state* s, const void* G, const void* R, const double* W, const double* q) {
  if (!s || !G || !R || !W || !q) return fail(CIS_E_INVALID_ARG, "NULL argument");
  const int64_t nc = s->mesh->nc, nv = s->dvs->n;
  size_t pb = (size_t)nc * nv * (s->precision == CIS_FP64 ? 8 : 4);
  HIP_TRY(hipMemcpyAsync(s->buf.G, G, pb, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(s->buf.R, R, pb, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(s->buf.W, W, 6 * nc * sizeof(double), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(s->buf.q, q, 6 * nc * sizeof(double), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CIS_OK;
}

cis_status cis_state_get(cis_state* s, void* G, void* R, double* W, double* q) {
  if (!s) return fail(CIS_E_INVALID_ARG, "state is NULL");
  const int64_t nc = s->mesh->nc, nv = s->dvs->n;
  size_t pb = (size_t)nc * nv * (s->precision == CIS_FP64 ? 8 : 4);
  if (G) HIP_TRY(hipMemcpyAsync(G, s->buf.G, pb, hipMemcpyDeviceToHost, s->stream));
  if (R) HIP_TRY(hipMemcpyAsync(R, s->buf.R, pb, hipMemcpyDeviceToHost, s->stream));
  if (W) HIP_TRY(hipMemcpyAsync(W, s->buf.W, 6 * nc * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  if (q) HIP_TRY(hipMemcpyAsync(q, s->buf.q, 6 * nc * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CIS_OK;
}

cis_status cis_iterate(cis_state* s, int32_t n_iter, double* res_hist) {
  if (!s) return fail(CIS_E_INVALID_ARG, "state is NULL");
  if (n_iter < 0) return fail(CIS_E_INVALID_ARG, "n_iter < 0");
  if (n_iter == 0) return CIS_OK;
  if (n_iter > s->res_cap) {
    double* nr = nullptr;
    HIP_TRY(hipMalloc((void**)&nr, 6 * (size_t)n_iter * sizeof(double)));
    for (auto& p : s->owned)
      if (p == (void*)s->work.res) {
        (void)hipStreamSynchronize(s->stream);
        (void)hipFree(p);
        p = (void*)nr;
      }
    s->work.res = nr;
    s->res_cap = n_iter;
  }
  std::vector<hipEvent_t> ev;
  if (s->profile) {
    ev.resize(7 * (size_t)n_iter, nullptr);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  }
  auto mark = [&](int32_t it, int k) {
    if (s->profile) (void)hipEventRecord(ev[7 * (size_t)it + k], s->stream);
  };
  cis_status st = enqueue_iterations(s, s->work, n_iter, mark);
  if (s->profile) {
    const cis_mesh* m = s->mesh;
    (void)hipStreamSynchronize(s->stream);
    const int64_t nmac = (int64_t)sweep_sequence(m->color_off.data(), m->n_colors, s->num.n_macro).size();
    const int64_t nmic = (int64_t)sweep_sequence(m->color_off.data(), m->n_colors, s->num.n_micro).size();
    const int64_t per_it[6] = {1, 1, 3 + nmac, 1, nmic, 3};
    for (int32_t it = 0; it < n_iter; ++it)
      for (int k = 0; k < 6; ++k) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev[7 * (size_t)it + k], ev[7 * (size_t)it + k + 1]);
        s->prof_ms[k] += ms;
        s->prof_launch[k] += per_it[k];
      }
    for (auto& e : ev) (void)hipEventDestroy(e);
  }
  if (st != CIS_OK) return st;
  return finish_iterations(s, s->work, n_iter, res_hist);
}

cis_status cis_iterate_noalloc(cis_state* s, int32_t n_iter, double* res_hist) {
  if (!s) return fail(CIS_E_INVALID_ARG, "state is NULL");
  if (n_iter < 0 || n_iter > kNoAllocMaxIter)
    return fail(CIS_E_INVALID_ARG, "n_iter must be in 0.." + std::to_string(kNoAllocMaxIter) +
                                       " for cis_iterate_noalloc (its residual history lives in a fixed device array)");
  if (n_iter == 0) return CIS_OK;
  double* sp = nullptr;
  cis_status st = scratch_of_device(s->device, &sp);
  if (st != CIS_OK) return st;
  // the state's work arrays, with the residual partials, the history and the flags in this device's scratch
  Work w = s->work;
  w.flag = reinterpret_cast<int32_t*>(sp);
  w.respart = sp + kScratchFlagDoubles;
  w.res = sp + kScratchFlagDoubles + kScratchPartDoubles;
  st = enqueue_iterations(s, w, n_iter, [](int32_t, int) {});
  if (st != CIS_OK) return st;
  return finish_iterations(s, w, n_iter, res_hist);
}

cis_status cis_residual(cis_state* s, void* FG, void* FR, double* Fmac) {
  if (!s || !FG || !FR) return fail(CIS_E_INVALID_ARG, "NULL argument");
  cis_status st = dispatch(s, [&](auto* tp) {
    using T = std::remove_pointer_t<decltype(tp)>;
    launch_recon<T>(s->dev, s->buf, s->stream);
    launch_face<T>(s->dev, s->buf, s->work, s->stream);
    launch_residual<T>(s->dev, s->buf, s->work, FG, FR, 1, s->stream);
    launch_macro_flux_cells(s->dev, s->work, s->stream);
    return device_check("residual");
  });
  if (st != CIS_OK) return st;
  if (Fmac) HIP_TRY(hipMemcpyAsync(Fmac, s->work.Fmac, 6 * s->mesh->nc * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CIS_OK;
}

cis_status cis_moments(cis_state* s, double* W, double* q) { return cis_state_get(s, nullptr, nullptr, W, q); }

cis_status cis_wall_heat_flux(cis_state* s, int32_t tag, double* Q) {
  if (!s || !Q) return fail(CIS_E_INVALID_ARG, "NULL argument");
  const cis_mesh* m = s->mesh;
  cis_status st = dispatch(s, [&](auto* tp) {
    using T = std::remove_pointer_t<decltype(tp)>;
    launch_recon<T>(s->dev, s->buf, s->stream);
    launch_face<T>(s->dev, s->buf, s->work, s->stream);
    return device_check("wall_heat_flux");
  });
  if (st != CIS_OK) return st;
  std::vector<double> fm(6 * m->nf);
  HIP_TRY(hipMemcpyAsync(fm.data(), s->work.face_mac, fm.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  double acc = 0.0;
  for (int64_t f = 0; f < m->nf; ++f)
    if (m->face_cell[2 * f + 1] < 0 && m->face_tag[f] == tag) acc += fm[6 * f + 4];
  *Q = acc;
  return CIS_OK;
}

cis_status cis_wall_loads(cis_state* s, int32_t tag, int64_t* n_faces, cis_wall_face* faces, double* force,
                          double* heat) {
  if (!s) return fail(CIS_E_INVALID_ARG, "state is NULL");
  std::vector<cis_wall_face> wf;
  double F[3], Q;
  cis_status st = wall_faces(s, tag, wf, F, &Q);
  if (st != CIS_OK) return st;
  if (faces) std::copy(wf.begin(), wf.end(), faces);
  if (n_faces) *n_faces = (int64_t)wf.size();
  if (force)
    for (int d = 0; d < 3; ++d) force[d] = F[d];
  if (heat) *heat = Q;
  return CIS_OK;
}

cis_status cis_wall_coefficients_of_loads(const cis_wall_face* faces, int64_t n_faces, double R,
                                          const cis_wall_ref* ref, cis_wall_coef* coef, cis_wall_totals* totals) {
  if ((n_faces > 0 && !faces) || n_faces < 0 || !ref) return fail(CIS_E_INVALID_ARG, "NULL argument or bad count");
  const double* U = ref->U_inf;
  const double Um = std::sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
  if (!(ref->rho_inf > 0.0) || !(Um > 0.0) || !std::isfinite(Um) || !(ref->T_inf > 0.0) || !(R > 0.0) ||
      !(ref->A_ref >= 0.0) || (ref->A_ref > 0.0 && !(ref->L_ref > 0.0)) || !finite_all(ref->x_ref, 3) ||
      !finite_all(ref->lift_dir, 3))
    return fail(CIS_E_INVALID_ARG, "reference values out of range");
  const double qd = 0.5 * ref->rho_inf * Um * Um;  // free-stream dynamic pressure
  const double p_inf = ref->rho_inf * R * ref->T_inf;
  double F[3] = {0.0, 0.0, 0.0}, M[3] = {0.0, 0.0, 0.0}, Q = 0.0;
  for (int64_t f = 0; f < n_faces; ++f) {
    const cis_wall_face& w = faces[f];
    const double tmag = std::sqrt(w.tau[0] * w.tau[0] + w.tau[1] * w.tau[1] + w.tau[2] * w.tau[2]);
    if (coef) {
      coef[f].Cp = (w.p - p_inf) / qd;    // Eq. 70
      coef[f].Ctau = tmag / qd;           // Eq. 71
      coef[f].Ch = w.q / (qd * Um);       // Eq. 72
    }
    double fa[3], r[3];
    for (int d = 0; d < 3; ++d) {
      fa[d] = w.area * (w.p * w.n[d] + w.tau[d]);
      r[d] = w.x[d] - ref->x_ref[d];
      F[d] += fa[d];
    }
    M[0] += r[1] * fa[2] - r[2] * fa[1];
    M[1] += r[2] * fa[0] - r[0] * fa[2];
    M[2] += r[0] * fa[1] - r[1] * fa[0];
    Q += w.area * w.q;
  }
  if (!totals) return CIS_OK;
  cis_wall_totals& t = *totals;
  std::memset(&t, 0, sizeof(t));
  for (int d = 0; d < 3; ++d) {
    t.force[d] = F[d];
    t.moment[d] = M[d];
  }
  t.heat = Q;
  // drag along U_inf; lift along the part of lift_dir normal to it (default e_z, or e_y when U_inf is along z)
  double eD[3] = {U[0] / Um, U[1] / Um, U[2] / Um}, eL[3];
  const bool dflt = ref->lift_dir[0] == 0.0 && ref->lift_dir[1] == 0.0 && ref->lift_dir[2] == 0.0;
  auto project = [&](const double* v) {
    const double a = v[0] * eD[0] + v[1] * eD[1] + v[2] * eD[2];
    for (int d = 0; d < 3; ++d) eL[d] = v[d] - a * eD[d];
    return std::sqrt(eL[0] * eL[0] + eL[1] * eL[1] + eL[2] * eL[2]);
  };
  const double ez[3] = {0.0, 0.0, 1.0}, ey[3] = {0.0, 1.0, 0.0};
  double len = project(dflt ? ez : ref->lift_dir);
  if (dflt && len < 1e-12) len = project(ey);
  if (!(len > 1e-12)) return fail(CIS_E_INVALID_ARG, "lift direction is parallel to U_inf");
  for (int d = 0; d < 3; ++d) {
    eL[d] /= len;
    t.e_drag[d] = eD[d];
    t.e_lift[d] = eL[d];
  }
  if (ref->A_ref > 0.0) {
    const double fs = 1.0 / (qd * ref->A_ref), ms = fs / ref->L_ref;
    for (int d = 0; d < 3; ++d) {
      t.CF[d] = F[d] * fs;
      t.CM[d] = M[d] * ms;
    }
    t.Cd = t.CF[0] * eD[0] + t.CF[1] * eD[1] + t.CF[2] * eD[2];
    t.Cl = t.CF[0] * eL[0] + t.CF[1] * eL[1] + t.CF[2] * eL[2];
    const double ep[3] = {eL[1] * eD[2] - eL[2] * eD[1], eL[2] * eD[0] - eL[0] * eD[2], eL[0] * eD[1] - eL[1] * eD[0]};
    t.Cm = t.CM[0] * ep[0] + t.CM[1] * ep[1] + t.CM[2] * ep[2];
    t.CQ = Q * fs / Um;
  }
  return CIS_OK;
}

cis_status cis_wall_coefficients(cis_state* s, int32_t tag, const cis_wall_ref* ref, int64_t* n_faces,
                                 cis_wall_coef* coef, cis_wall_totals* totals) {
  if (!s || !ref) return fail(CIS_E_INVALID_ARG, "NULL argument");
  std::vector<cis_wall_face> wf;
  double F[3], Q;
  cis_status st = wall_faces(s, tag, wf, F, &Q);
  if (st != CIS_OK) return st;
  if (n_faces) *n_faces = (int64_t)wf.size();
  return cis_wall_coefficients_of_loads(wf.data(), (int64_t)wf.size(), s->gas.R, ref, coef, totals);
}

cis_status cis_profile_enable(cis_state* s, int32_t enable) {
  if (!s) return fail(CIS_E_INVALID_ARG, "state is NULL");
  s->profile = enable != 0;
  for (int k = 0; k < 6; ++k) {
    s->prof_ms[k] = 0.0;
    s->prof_launch[k] = 0;
  }
  return CIS_OK;
}

cis_status cis_profile_read(cis_state* s, double* ms, int64_t* launches) {
  if (!s) return fail(CIS_E_INVALID_ARG, "state is NULL");
  for (int k = 0; k < 6; ++k) {
    if (ms) ms[k] = s->prof_ms[k];
    if (launches) launches[k] = s->prof_launch[k];
  }
  return CIS_OK;
}

cis_status cis_debug_stage(cis_state* s, int32_t which, double* out) {
  if (!s || !out) return fail(CIS_E_INVALID_ARG, "NULL argument");
  const int64_t nc = s->mesh->nc;
  if (which == 0 || which == 1 || which == 2) {
    const double* src = which == 0 ? s->work.dW : which == 1 ? s->work.Wt : s->work.Fmac;
    HIP_TRY(hipMemcpyAsync(out, src, 6 * nc * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return CIS_OK;
  }
  if (which == 3) {
    std::vector<double> eq(ER * nc);
    HIP_TRY(hipMemcpyAsync(eq.data(), s->work.eq, eq.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int64_t i = 0; i < nc; ++i) out[i] = eq[ER * i + 7];
    return CIS_OK;
  }
  return fail(CIS_E_INVALID_ARG, "unknown stage");
}

cis_status cis_state_set_bc(cis_state* s, const cis_bc* bc, int32_t n_bc) {
  if (!s || (n_bc > 0 && !bc)) return fail(CIS_E_INVALID_ARG, "NULL argument");
  if ((size_t)n_bc != s->bcs.size()) return fail(CIS_E_INVALID_ARG, "n_bc differs from the state's");
  for (int b = 0; b < n_bc; ++b) {
    if (bc[b].tag != s->bcs[b].tag || bc[b].kind != s->bcs[b].kind)
      return fail(CIS_E_INVALID_ARG, "tags and kinds must match the state's");
    if (!(bc[b].T > 0.0) || (bc[b].kind == CIS_BC_FARFIELD && !(bc[b].rho > 0.0)) || !finite_all(bc[b].U, 3))
      return fail(CIS_E_INVALID_ARG, "bc values out of range");
  }
  std::vector<double> bct(BCW * std::max(n_bc, 1), 0.0);
  for (int b = 0; b < n_bc; ++b) {
    double* p = &bct[BCW * b];
    p[0] = bc[b].kind;
    p[1] = bc[b].rho;
    for (int d = 0; d < 3; ++d) p[2 + d] = bc[b].U[d];
    p[5] = bc[b].T;
  }
  HIP_TRY(hipMemcpyAsync(s->d_bc, bct.data(), bct.size() * sizeof(double), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->bcs.assign(bc, bc + n_bc);
  return CIS_OK;
}

cis_status cis_steady_residual(cis_state* s, int32_t wall_tag, double* rG, double* rR, double* rW, double* rq,
                               double* J) {
  if (!s || !rG || !rR || !rW || !rq) return fail(CIS_E_INVALID_ARG, "NULL argument");
  if (s->num.limiter == 4) return fail(CIS_E_UNSUPPORTED, "limiter 4 updates its values: use limiter 3 (stored values)");
  if (s->precision != CIS_FP64) return fail(CIS_E_UNSUPPORTED, "the steady residual is FP64 only");
  launch_recon<double>(s->dev, s->buf, s->stream);
  launch_face<double>(s->dev, s->buf, s->work, s->stream);
  launch_residual<double>(s->dev, s->buf, s->work, rG, rR, 1, s->stream);
  launch_cell_steady(s->dev, s->buf, rG, rR, rW, rq, s->stream);
  cis_status st = device_check("steady_residual");
  if (st != CIS_OK) return st;
  if (J) return objective_from_faces(s, slot_of(s, wall_tag), J);
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CIS_OK;
}

cis_status cis_residual_vjp(cis_state* s, const double* vG, const double* vR, const double* vW, const double* vq,
                            double cJ, int32_t wall_tag, int32_t ff_tag, double* gG, double* gR, double* gW,
                            double* gq, double* gp) {
  if (!s || !gG || !gR || !gW || !gq) return fail(CIS_E_INVALID_ARG, "NULL argument");
  const bool anyv = vG || vR || vW || vq, allv = vG && vR && vW && vq;
  if (anyv && !allv) return fail(CIS_E_INVALID_ARG, "vG, vR, vW, vq must be all set or all NULL");
  if (!std::isfinite(cJ)) return fail(CIS_E_INVALID_ARG, "non-finite cJ");
  if (s->precision != CIS_FP64) return fail(CIS_E_UNSUPPORTED, "the VJP is FP64 only");
  if (s->num.limiter == 4) return fail(CIS_E_UNSUPPORTED, "limiter 4 updates its values: use limiter 3 (stored values)");
  AdjSlots sl;
  cis_status st = adj_slots(s, wall_tag, ff_tag, cJ != 0.0, &sl);
  if (st != CIS_OK) return st;
  AdjArgs a{vG, vR, vW, vq, cJ, sl.j, sl.w, sl.f, gG, gR, gW, gq, s->work.gpf};
  launch_vjp(s->dev, s->buf, a, s->stream);
  st = device_check("residual_vjp");
  if (st != CIS_OK) return st;
  if (gp) return sum_gp(s, gp);
  HIP_TRY(hipStreamSynchronize(s->stream));
  return CIS_OK;
}

cis_status cis_adjoint_required_bytes(const cis_state* s, int32_t restart, int64_t* bytes) {
  if (!s || !bytes) return fail(CIS_E_INVALID_ARG, "NULL argument");
  if (restart < 1 || restart > 1000) return fail(CIS_E_INVALID_ARG, "restart must be in 1..1000");
  *bytes = adjoint_doubles(s, restart) * (int64_t)sizeof(double);
  return CIS_OK;
}

cis_status cis_adjoint_solve(cis_state* s, int32_t wall_tag, int32_t ff_tag, int32_t restart, int32_t max_iter,
                             double rtol, int32_t precond_pairs, int32_t macro_pairs, void* work,
                             int64_t work_bytes, double* lam, double* dJdp, double* J, cis_adjoint_info* info) {
  if (!s || !work || !lam || !dJdp) return fail(CIS_E_INVALID_ARG, "NULL argument");
  if (s->precision != CIS_FP64) return fail(CIS_E_UNSUPPORTED, "the adjoint is FP64 only");
  if (s->num.limiter == 4) return fail(CIS_E_UNSUPPORTED, "limiter 4 updates its values: use limiter 3 (stored values)");
  if (restart < 1 || restart > 1000 || max_iter < 0 || !(rtol > 0.0) || precond_pairs < 0 || precond_pairs > 64 ||
      macro_pairs < 0 || macro_pairs > 200)
    return fail(CIS_E_INVALID_ARG, "restart, max_iter, rtol, precond_pairs or macro_pairs out of range");
  if (work_bytes < adjoint_doubles(s, restart) * (int64_t)sizeof(double))
    return fail(CIS_E_INVALID_ARG, "work buffer smaller than cis_adjoint_required_bytes");
  AdjSlots sl;
  cis_status st = adj_slots(s, wall_tag, ff_tag, true, &sl);
  if (st != CIS_OK) return st;
  const int m = restart;
  const int64_t N = 2 * s->mesh->nc * s->dvs->n + 12 * s->mesh->nc;
  double* V = (double*)work;               // [m+1][N] Krylov basis
  double* b = V + (int64_t)(m + 1) * N;    // right-hand side dJ/dx
  double* z = b + N;                       // preconditioned vector / update
  double* part = z + N;                    // [m+1][dot_partials()]
  double* hdev = part + (int64_t)(m + 2) * dot_partials();
  double* ptmp = hdev + (m + 2);           // block preconditioner: a full-length vector and per-cell scratch
  double* pcell = ptmp + N;
  hipStream_t q = s->stream;
  auto dots = [&](const double* Vb, int nvec, const double* w, double* host) {
    return dev_dots(s, Vb, N, nvec, w, part, hdev, host);
  };
  auto precond = [&](const double* in, double* out) {
    if (macro_pairs > 0)
      launch_adj_block_precond(s->dev, s->buf, in, out, ptmp, pcell, s->mesh->color_off.data(), s->mesh->n_colors,
                               precond_pairs, macro_pairs, q);
    else if (precond_pairs == 0)
      launch_precond(s->dev, s->buf, in, out, q);
    else
      launch_adj_sweeps(s->dev, s->buf, in, out, s->mesh->color_off.data(), s->mesh->n_colors, precond_pairs, q);
  };
  // right-hand side and the explicit parameter dependence of J
  double gpJ[3], gpL[3] = {0.0, 0.0, 0.0};
  run_vjp(s, nullptr, 1.0, sl, b);
  if ((st = device_check("adjoint rhs")) != CIS_OK) return st;
  if ((st = sum_gp(s, gpJ)) != CIS_OK) return st;
  double bn2;
  if ((st = dots(b, 1, b, &bn2)) != CIS_OK) return st;
  const double bnorm = std::sqrt(bn2);
  launch_axpby(N, 0.0, b, 0.0, lam, q);
  int32_t iters = 0;
  double beta = bnorm;
  launch_axpby(N, 1.0, b, 0.0, V, q);  // r = b - A*0
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m), h(m + 1), h2(m + 1);
  bool done = bnorm == 0.0;
  while (!done && iters < max_iter) {
    launch_axpby(N, 1.0 / beta, V, 0.0, V, q);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int jend = 0;
    for (int j = 0; j < m && iters < max_iter; ++j) {
      double* vj = V + (int64_t)j * N;
      double* w = V + (int64_t)(j + 1) * N;
      precond(vj, z);
      run_vjp(s, z, 0.0, sl, w);
      // classical Gram-Schmidt, twice
      if ((st = dots(V, j + 1, w, h.data())) != CIS_OK) return st;
      launch_gemv_sub(V, N, j + 1, hdev, w, q);
      if ((st = dots(V, j + 1, w, h2.data())) != CIS_OK) return st;
      launch_gemv_sub(V, N, j + 1, hdev, w, q);
      for (int i = 0; i <= j; ++i) h[i] += h2[i];
      double hn2;
      if ((st = dots(w, 1, w, &hn2)) != CIS_OK) return st;
      const double hn = std::sqrt(hn2);
      if (hn > 0.0) launch_axpby(N, 1.0 / hn, w, 0.0, w, q);
      // Givens rotations on column j
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
      }
      const double r = std::hypot(h[j], hn);
      cs[j] = r > 0.0 ? h[j] / r : 1.0;
      sn[j] = r > 0.0 ? hn / r : 0.0;
      h[j] = r;
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      ++iters;
      jend = j + 1;
      if (std::fabs(gv[j + 1]) <= rtol * bnorm || hn == 0.0) break;
    }
    // y = H^-1 g, lam += M^-1 (V y)
    for (int i = jend - 1; i >= 0; --i) {
      double t = gv[i];
      for (int k = i + 1; k < jend; ++k) t -= H[(size_t)i * m + k] * y[k];
      y[i] = t / H[(size_t)i * m + i];
    }
    for (int i = 0; i < jend; ++i) y[i] = -y[i];
    HIP_TRY(hipMemcpyAsync(hdev, y.data(), jend * sizeof(double), hipMemcpyHostToDevice, q));
    launch_axpby(N, 0.0, z, 0.0, z, q);
    launch_gemv_sub(V, N, jend, hdev, z, q);
    precond(z, V + (int64_t)m * N);
    launch_axpby(N, 1.0, V + (int64_t)m * N, 1.0, lam, q);
    // true residual r = b - A lam, and lam^T dR/dp
    run_vjp(s, lam, 0.0, sl, V);
    if ((st = device_check("adjoint iteration")) != CIS_OK) return st;
    if ((st = sum_gp(s, gpL)) != CIS_OK) return st;
    launch_axpby(N, 1.0, b, -1.0, V, q);
    double r2;
    if ((st = dots(V, 1, V, &r2)) != CIS_OK) return st;
    beta = std::sqrt(r2);
    done = beta <= rtol * bnorm || beta == 0.0;
  }
  for (int k = 0; k < 3; ++k) dJdp[k] = gpJ[k] - gpL[k];
  if (info) {
    info->iterations = iters;
    info->converged = done ? 1 : 0;
    info->rel_residual = bnorm > 0.0 ? beta / bnorm : 0.0;
  }
  if (J) {
    launch_recon<double>(s->dev, s->buf, q);
    launch_face<double>(s->dev, s->buf, s->work, q);
    if ((st = device_check("objective")) != CIS_OK) return st;
    return objective_from_faces(s, sl.j, J);
  }
  HIP_TRY(hipStreamSynchronize(q));
  return CIS_OK;
}

}  // extern "C"
