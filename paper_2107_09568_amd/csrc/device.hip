// Device state of a plan: uploads of the host set-up, the table copies used by
// the precision modes, the device CSR structure, the degeneracy check and the
// CSR matrix-vector product.
#include <cstring>
#include <string>

#include "device_common.h"

namespace igamt {

template <typename T>
static igamt_status dev_upload(T **dst, const T *src, size_t count) {
  if (count == 0) count = 1;
  IGAMT_HIP(hipMalloc((void **)dst, count * sizeof(T)));
  if (src) IGAMT_HIP(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return IGAMT_OK;
}

#define UP(dst, vec) \
  do { igamt_status s_ = dev_upload(&(dst), (vec).data(), (vec).size()); if (s_) return s_; } while (0)

static __global__ void fill_i32(int32_t *p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

igamt_status ensure_device(igamt_plan *P) {
  DevicePtrs &d = P->dev;
  int cur = 0;
  IGAMT_HIP(hipGetDevice(&cur));
  if (d.ready) {
    if (cur != d.device) { set_error("plan used on a different device than it was set up on"); return IGAMT_ESTATE; }
    return IGAMT_OK;
  }
  d.device = cur;
  for (int k = 0; k < 3; ++k) {
    UP(d.macro_knots[k], P->kM[k]);
    UP(d.box_a[k], P->box_a[k]);
    UP(d.box_h[k], P->box_h[k]);
    UP(d.tile_knots[k], P->kT[k]);
    UP(d.dir_pairs[k], P->dir[k].pairs);
    UP(d.dir_off[k], P->dir[k].off);
    UP(d.dir_pre[k], P->dir[k].pre);
    UP(d.dir_lo[k], P->dir[k].lo);
    UP(d.ctrl_lo[k], P->ctrl_lo[k]);
    UP(d.ctrl_tiles_off[k], P->ctrl_tiles_off[k]);
    UP(d.ctrl_tiles[k], P->ctrl_tiles[k]);
  }
  UP(d.macro_ctrl, P->ctrlM);
  if (!P->wM.empty()) UP(d.macro_w, P->wM);
  UP(d.tile_ctrl, P->ctrlT);
  UP(d.tile_grev, P->grevT);
  UP(d.fit_x, P->fit_x);
  UP(d.fit_P, P->fit_P);
  UP(d.fit_P3, P->fit_P3);
  UP(d.gauss_x, P->gauss_x);
  UP(d.gauss_w, P->gauss_w);
  UP(d.pairs, P->pairs);
  UP(d.pair_lut, P->pair_lut);
  UP(d.mirror_perm, P->mirror_perm);
  UP(d.pair_desc, P->pair_desc);
  IGAMT_HIP(hipMalloc((void **)&d.flag, 4 * sizeof(int32_t)));
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, 0, d.flag, 4, INT32_MAX);
  IGAMT_LAUNCH_CHECK();
  const int64_t MK = P->Mp * P->Kp;
  IGAMT_HIP(hipMalloc((void **)&d.table, MK * sizeof(double)));
  const int64_t MKt = transposed_rows(P) * P->Mp;   // rows past Kp stay zero
  IGAMT_HIP(hipMalloc((void **)&d.table_t, MKt * sizeof(double)));
  IGAMT_HIP(hipMemset(d.table_t, 0, MKt * sizeof(double)));
  IGAMT_HIP(hipMalloc((void **)&d.table_f32, MK * sizeof(float)));
  IGAMT_HIP(hipMalloc((void **)&d.table_t_f32, MKt * sizeof(float)));
  IGAMT_HIP(hipMemset(d.table_t_f32, 0, MKt * sizeof(float)));
  IGAMT_HIP(hipMalloc((void **)&d.table_bf, 2 * MK * sizeof(uint16_t)));
  IGAMT_HIP(hipMalloc((void **)&d.table_h, 2 * MK * sizeof(uint16_t)));
  IGAMT_HIP(hipMalloc((void **)&d.table_h_scale, P->Mp * sizeof(float)));
  IGAMT_HIP(hipDeviceSynchronize());
  // the allocation-free volume entry point reports a failed lookup itself; nothing else needs it
  (void)volume_scratch_setup(cur);
  d.ready = true;
  return IGAMT_OK;
}

void free_device(igamt_plan *P) {
  DevicePtrs &d = P->dev;
  if (!d.ready) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(d.device);
  (void)hipDeviceSynchronize();
  void *ptrs[] = {d.macro_ctrl, d.macro_w, d.fit_x, d.fit_P, d.fit_P3, d.tile_ctrl, d.tile_grev, d.gauss_x, d.gauss_w, d.pairs, d.pair_lut,
                  d.flag, d.table, d.table_t, d.table_f32, d.table_t_f32, d.table_bf, d.table_h,
                  d.table_h_scale, d.point_data, d.mirror_perm, d.pair_desc,
                  d.batch_points, d.load_table, d.apply_rec, d.volume_data, d.eproj_buf};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (int k = 0; k < 3; ++k) {
    void *q[] = {d.macro_knots[k], d.box_a[k], d.box_h[k], d.tile_knots[k], d.dir_pairs[k], d.dir_off[k],
                 d.dir_pre[k], d.dir_lo[k], d.ctrl_lo[k], d.ctrl_tiles_off[k], d.ctrl_tiles[k]};
    for (void *p : q)
      if (p) (void)hipFree(p);
  }
  (void)hipSetDevice(cur);
  d = DevicePtrs();
  P->batch_points_cap = 0;
  P->load_table_ready = false;
  P->volume_ready = false;
}

igamt_status upload_tile_ctrl(igamt_plan *P) {
  IGAMT_HIP(hipMemcpy(P->dev.tile_ctrl, P->ctrlT.data(), P->ctrlT.size() * sizeof(double), hipMemcpyHostToDevice));
  return IGAMT_OK;
}

// A tile control point on the tile boundary that is not at its Greville position breaks the
// gluing of neighbouring tiles: the smallest such point index goes to flag[2].
static __global__ void tile_boundary_kernel(const double *__restrict__ ctrl, const double *__restrict__ grev, int nx,
                                            int ny, int nz, int32_t *flag) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nx * ny * nz) return;
  const int i = id % nx, j = (id / nx) % ny, k = id / (nx * ny);
  if (!(i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1)) return;
  const double e = fabs(ctrl[3 * id] - grev[i]) + fabs(ctrl[3 * id + 1] - grev[nx + j]) +
                   fabs(ctrl[3 * id + 2] - grev[nx + ny + k]);
  if (!(e <= 1e-12)) atomicMin(flag + 2, id);
}

// The device copy is the current one once ensure_device has run (it is the only upload from the
// host copy P->ctrlM); a device-side set leaves P->ctrlM behind, and nothing reads it afterwards.
igamt_status upload_macro_ctrl(igamt_plan *P, const double *ctrl, int on_device, void *stream) {
  const int64_t n = 3LL * P->nM[0] * P->nM[1] * P->nM[2];
  hipStream_t s = (hipStream_t)stream;
  if (on_device) {
    IGAMT_HIP(hipMemcpyAsync(P->dev.macro_ctrl, ctrl, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(ctrl[i])) { set_error("non-finite macro control point"); return IGAMT_EINVAL; }
    std::memcpy(P->ctrlM.data(), ctrl, n * sizeof(double));
    IGAMT_HIP(hipMemcpyAsync(P->dev.macro_ctrl, P->ctrlM.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
    IGAMT_HIP(hipStreamSynchronize(s));
  }
  return IGAMT_OK;
}

// One block per table row: FP32 copy, bfloat16 hi/lo split, float16 hi/lo split
// with a power-of-two row scale (padding rows/columns are zero and stay zero).
static __global__ __launch_bounds__(256) void table_copies_kernel(const int32_t *gate, const double *__restrict__ T, int64_t Kp,
                                                                  float *__restrict__ T32, uint16_t *__restrict__ Tbf,
                                                                  uint16_t *__restrict__ Th, float *__restrict__ hscale,
                                                                  int64_t MK) {
  if (gate && *gate == 0) return;
  const int64_t row = blockIdx.x;
  const double *r = T + row * Kp;
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t k = threadIdx.x; k < Kp; k += 256) m = fmax(m, fabs(r[k]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double sc = f16_scale_for(red[0]);
  if (threadIdx.x == 0) hscale[row] = (float)(1.0 / sc);
  for (int64_t k = threadIdx.x; k < Kp; k += 256) {
    const double x = r[k];
    T32[row * Kp + k] = (float)x;
    uint16_t hi, lo;
    split_bf16(x, hi, lo);
    Tbf[row * Kp + k] = hi;
    Tbf[MK + row * Kp + k] = lo;
    split_f16(x * sc, hi, lo);
    Th[row * Kp + k] = hi;
    Th[MK + row * Kp + k] = lo;
  }
}

static __global__ void transpose_kernel(const int32_t *gate, const double *__restrict__ T, int64_t Mp, int64_t Kp,
                                        double *__restrict__ Tt, float *__restrict__ Tt32) {
  if (gate && *gate == 0) return;
  __shared__ double tile[32][33];
  const int64_t k0 = (int64_t)blockIdx.x * 32, m0 = (int64_t)blockIdx.y * 32;
  for (int j = threadIdx.y; j < 32; j += 8) tile[j][threadIdx.x] = T[(m0 + j) * Kp + k0 + threadIdx.x];
  __syncthreads();
  for (int j = threadIdx.y; j < 32; j += 8) {
    const double v = tile[threadIdx.x][j];
    Tt[(k0 + j) * Mp + m0 + threadIdx.x] = v;
    Tt32[(k0 + j) * Mp + m0 + threadIdx.x] = (float)v;
  }
}

igamt_status derive_table_copies(igamt_plan *P, void *stream, const int32_t *gate) {
  hipStream_t s = (hipStream_t)stream;
  DevicePtrs &d = P->dev;
  hipLaunchKernelGGL(table_copies_kernel, dim3((unsigned)P->Mp), dim3(256), 0, s, gate, d.table, (int64_t)P->Kp,
                     d.table_f32, d.table_bf, d.table_h, d.table_h_scale, P->Mp * P->Kp);
  IGAMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)(P->Kp / 32), (unsigned)(P->Mp / 32)), dim3(32, 8), 0, s,
                     gate, d.table, (int64_t)P->Mp, (int64_t)P->Kp, d.table_t, d.table_t_f32);
  IGAMT_LAUNCH_CHECK();
  P->tables_ready = true;
  return IGAMT_OK;
}

static __global__ void fill_f64(double *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

static __global__ void pad_copy_kernel(const double *__restrict__ src, int64_t rows, int64_t K, double *__restrict__ dst,
                                       int64_t Kp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * K) return;
  const int64_t r = i / K, c = i % K;
  dst[r * Kp + c] = src[i];
}

static __global__ void unpad_copy_kernel(const double *__restrict__ src, int64_t rows, int64_t K, int64_t Kp,
                                         double *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * K) return;
  const int64_t r = i / K, c = i % K;
  dst[i] = src[r * Kp + c];
}

// ---- CSR structure on the device -------------------------------------------
struct GridArgs {
  const Pair1D *p[3];
  const int64_t *pre[3];
  int64_t E[3];
  int NG[3];
};

static GridArgs grid_args(const igamt_plan *P) {
  GridArgs g;
  for (int k = 0; k < 3; ++k) {
    g.p[k] = P->dev.dir_pairs[k];
    g.pre[k] = P->dev.dir_pre[k];
    g.E[k] = (int64_t)P->dir[k].pairs.size();
    g.NG[k] = P->dir[k].NG;
  }
  return g;
}

static __global__ __launch_bounds__(256) void csr_cols_kernel(GridArgs g, int32_t *__restrict__ col) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = g.E[0] * g.E[1] * g.E[2];
  if (idx >= total) return;
  const int64_t ex = idx % g.E[0];
  const int64_t r = idx / g.E[0];
  const int64_t ey = r % g.E[1], ez = r / g.E[1];
  const Pair1D X = g.p[0][ex], Y = g.p[1][ey], Z = g.p[2][ez];
  const int64_t SX = g.pre[0][g.NG[0]], SY = g.pre[1][g.NG[1]];
  const int64_t cx = g.pre[0][X.g + 1] - g.pre[0][X.g];
  const int64_t cy = g.pre[1][Y.g + 1] - g.pre[1][Y.g];
  const int64_t cz = g.pre[2][Z.g + 1] - g.pre[2][Z.g];
  const int64_t nnb = cx * cy * cz;
  const int64_t before = g.pre[2][Z.g] * SY * SX + cz * (g.pre[1][Y.g] * SX + cy * g.pre[0][X.g]);
  const int64_t rank = ((int64_t)Z.rank * cy + Y.rank) * cx + X.rank;
  const int64_t base = 9 * before + 3 * rank;
  const int64_t G2 = X.g2 + (int64_t)g.NG[0] * (Y.g2 + (int64_t)g.NG[1] * Z.g2);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) col[base + 3 * a * nnb + b] = (int32_t)(3 * G2 + b);
}

static __global__ __launch_bounds__(256) void csr_rowptr_kernel(GridArgs g, int64_t *__restrict__ row_ptr, int64_t nnz) {
  const int64_t G = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t NGt = (int64_t)g.NG[0] * g.NG[1] * g.NG[2];
  if (G > NGt) return;
  if (G == NGt) { row_ptr[3 * NGt] = nnz; return; }
  const int gx = (int)(G % g.NG[0]);
  const int gy = (int)((G / g.NG[0]) % g.NG[1]);
  const int gz = (int)(G / ((int64_t)g.NG[0] * g.NG[1]));
  const int64_t SX = g.pre[0][g.NG[0]], SY = g.pre[1][g.NG[1]];
  const int64_t cx = g.pre[0][gx + 1] - g.pre[0][gx];
  const int64_t cy = g.pre[1][gy + 1] - g.pre[1][gy];
  const int64_t cz = g.pre[2][gz + 1] - g.pre[2][gz];
  const int64_t nnb = cx * cy * cz;
  const int64_t before = g.pre[2][gz] * SY * SX + cz * (g.pre[1][gy] * SX + cy * g.pre[0][gx]);
  for (int a = 0; a < 3; ++a) row_ptr[3 * G + a] = 9 * before + 3 * a * nnb;
}

// ---- CSR SpMV ----------------------------------------------------------------
template <typename T>
static __global__ __launch_bounds__(256) void spmv_kernel(int64_t n, const int64_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci, const T *__restrict__ v,
                                                          const T *__restrict__ x, T *__restrict__ y) {
  // one wave per row, fixed-order reduction (deterministic)
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  T acc = 0;
  for (int64_t j = rp[row] + lane; j < rp[row + 1]; j += 64) acc += v[j] * x[ci[j]];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) y[row] = acc;
}

}  // namespace igamt

using namespace igamt;

extern "C" igamt_status igamt_set_macro_ctrl(igamt_plan *P, const double *ctrl, int32_t on_device, void *stream) {
  if (!P || !ctrl) { set_error("NULL argument"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  return upload_macro_ctrl(P, ctrl, on_device, stream);
}

extern "C" igamt_status igamt_tables_set(igamt_plan *P, const double *d_table, void *stream) {
  if (!P || !d_table) { set_error("NULL argument"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t MK = P->Mp * P->Kp;
  hipLaunchKernelGGL(fill_f64, dim3((unsigned)((MK + 255) / 256)), dim3(256), 0, s, P->dev.table, MK);
  IGAMT_LAUNCH_CHECK();
  const int64_t n = P->n_pairs * P->K;
  hipLaunchKernelGGL(pad_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_table, P->n_pairs,
                     (int64_t)P->K, P->dev.table, (int64_t)P->Kp);
  IGAMT_LAUNCH_CHECK();
  return derive_table_copies(P, stream);
}

extern "C" igamt_status igamt_tables_get(const igamt_plan *P, double *d_out, void *stream) {
  if (!P || !d_out) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (!P->dev.ready || !P->tables_ready) { set_error("tables not built"); return IGAMT_ESTATE; }
  const int64_t n = P->n_pairs * P->K;
  hipLaunchKernelGGL(unpad_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     P->dev.table, P->n_pairs, (int64_t)P->K, (int64_t)P->Kp, d_out);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

extern "C" igamt_status igamt_plan_csr_device(igamt_plan *P, int64_t *d_row_ptr, int32_t *d_col_idx, void *stream) {
  if (!P || !d_row_ptr || !d_col_idx) { set_error("NULL argument"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  GridArgs g = grid_args(P);
  const int64_t total = g.E[0] * g.E[1] * g.E[2];
  hipLaunchKernelGGL(csr_cols_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g, d_col_idx);
  IGAMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(csr_rowptr_kernel, dim3((unsigned)((P->n_global + 1 + 255) / 256)), dim3(256), 0, s, g,
                     d_row_ptr, P->nnz);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

extern "C" igamt_status igamt_set_tile_ctrl_device(igamt_plan *P, const double *d_ctrl, void *stream) {
  if (!P || !d_ctrl) { set_error("NULL argument"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  IGAMT_HIP(hipMemcpyAsync(P->dev.tile_ctrl, d_ctrl, 3 * P->nTt * sizeof(double), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(tile_boundary_kernel, dim3((unsigned)((P->nTt + 255) / 256)), dim3(256), 0, s, P->dev.tile_ctrl,
                     P->dev.tile_grev, P->nT[0], P->nT[1], P->nT[2], P->dev.flag);
  IGAMT_LAUNCH_CHECK();
  P->tables_ready = false;
  P->load_table_ready = false;
  P->volume_ready = false;
  return IGAMT_OK;
}

extern "C" igamt_status igamt_check(igamt_plan *P, void *stream, int64_t *bad_tile) {
  if (!P) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (bad_tile) *bad_tile = -1;
  if (!P->dev.ready) return IGAMT_OK;
  hipStream_t s = (hipStream_t)stream;
  IGAMT_HIP(hipStreamSynchronize(s));
  int32_t h[4];
  IGAMT_HIP(hipMemcpy(h, P->dev.flag, sizeof(h), hipMemcpyDeviceToHost));
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, P->dev.flag, 4, INT32_MAX);
  IGAMT_LAUNCH_CHECK();
  IGAMT_HIP(hipStreamSynchronize(s));
  if (h[0] != INT32_MAX) {
    if (bad_tile) *bad_tile = h[0];
    set_error("degenerate macro element (det J <= 0) at tile " + std::to_string(h[0]));
    return IGAMT_EDEGENERATE;
  }
  if (h[1] != INT32_MAX) {
    if (bad_tile) *bad_tile = h[1];
    set_error("reference tile map not positively oriented in micro element " + std::to_string(h[1]));
    return IGAMT_EDEGENERATE;
  }
  if (h[2] != INT32_MAX) {
    set_error("tile boundary control point " + std::to_string(h[2]) + " is not at its Greville position");
    return IGAMT_EINVAL;
  }
  return IGAMT_OK;
}

extern "C" igamt_status igamt_spmv(igamt_precision prec, int64_t n, const int64_t *rp, const int32_t *ci,
                                   const void *v, const void *x, void *y, void *stream) {
  if (!rp || !ci || !v || !x || !y || n < 0) { set_error("invalid argument"); return IGAMT_EINVAL; }
  if (n == 0) return IGAMT_OK;
  const dim3 grid((unsigned)((n + 3) / 4));
  hipStream_t s = (hipStream_t)stream;
  if (prec == IGAMT_F64)
    hipLaunchKernelGGL(spmv_kernel<double>, grid, dim3(256), 0, s, n, rp, ci, (const double *)v, (const double *)x,
                       (double *)y);
  else
    hipLaunchKernelGGL(spmv_kernel<float>, grid, dim3(256), 0, s, n, rp, ci, (const float *)v, (const float *)x,
                       (float *)y);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}
