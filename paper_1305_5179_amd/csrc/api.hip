// C ABI of librbf (declared in include/rbf.h): argument checks, the setup
// pipeline, the operator, the GMRES driver and the evaluation entry points.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>

#include "common.h"

namespace rbf {

// krylov.hip
int gm_max_restart();
size_t gm_state_bytes();
int64_t gm_partial_count(int64_t n);
void gm_start(const double* b, const double* y, double* r, int64_t n, void* V, bool f32, double* partial, int m,
              double tol_abs, void* state, hipStream_t s);
void gm_step(void* V, int64_t ldv, void* w, bool f32, int64_t n, int j, double* partial, void* state,
             hipStream_t s);
void gm_finish(const void* V, int64_t ldv, bool f32, double* x, int64_t n, void* state, hipStream_t s);
void to_f64(const float* x, double* y, int64_t n, hipStream_t s);
void gm_read(const void* state, int* k, int* done, int* breakdown, double* beta0, double* gk, hipStream_t s);
void gm_set_tol(void* state, double tol_abs, hipStream_t s);
const int* gm_done_flag(const void* state);
int gm_read_hessenberg(const void* state, int m, double* H, int* breakdown, hipStream_t s);

namespace {

thread_local std::string t_err = "no error";

int fail(Ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  t_err = msg;
  return code;
}

template <class F>
int guarded(Ctx* c, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return fail(c, e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(c, RBF_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(c, RBF_EDEVICE, e.what());
  }
}

// The library is built for gfx950 only.
// The architecture check runs once per device (hipGetDeviceProperties takes
// milliseconds); the verdict is kept for the life of the process.
int check_device(Ctx* c, int* dev_out) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0)
    return fail(c, RBF_EDEVICE, std::string("no HIP device available (") + hipGetErrorString(e) + ")");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(c, RBF_EDEVICE, "hipGetDevice failed");
  static std::mutex mu;
  static std::map<int, std::string> arch;   // device -> gcnArchName
  std::string name;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = arch.find(dev);
    if (it == arch.end()) {
      hipDeviceProp_t p;
      if (hipGetDeviceProperties(&p, dev) != hipSuccess) return fail(c, RBF_EDEVICE, "hipGetDeviceProperties failed");
      it = arch.emplace(dev, std::string(p.gcnArchName)).first;
    }
    name = it->second;
  }
  if (name.compare(0, 6, "gfx950") != 0) return fail(c, RBF_EDEVICE, "device " + name + " is not gfx950");
  *dev_out = dev;
  return RBF_OK;
}

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}


void drop_cycle_graph(Ctx* c) {
  if (c->cycle_exec) (void)hipGraphExecDestroy(c->cycle_exec);
  c->cycle_exec = nullptr;
  c->cycle_key.clear();
}

void free_ctx(Ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  SyncedRelease synced;   // the device is idle: the blocks may go to any stream
  drop_cycle_graph(c);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  c->capture_stream = nullptr;
  free_targets(c->centres);
  free_schwarz(c->schwarz);
  c->schwarz = nullptr;
  free_net(c->net);
  c->net = nullptr;
  for (void* p : {(void*)c->perm, (void*)c->keys, (void*)c->xs, (void*)c->xk, (void*)c->xpaper, (void*)c->cell_start,
                  (void*)c->cell_count, (void*)c->cell_map, (void*)c->cell_xyz, (void*)c->cell_sat, (void*)c->vin,
                  (void*)c->vout,
                  (void*)c->V, (void*)c->w, (void*)c->r, (void*)c->csol, (void*)c->bsort, (void*)c->partial,
                  (void*)c->state})
    dfree(p);
}

// Neighbour lattice for the centre bounding box (see the Lattice comment).
Lattice make_lattice(const double box[6], double cutoff) {
  Lattice L{};
  double ext[3], maxext = 0.0;
  for (int d = 0; d < 3; ++d) {
    ext[d] = box[3 + d] - box[d];
    maxext = std::max(maxext, ext[d]);
  }
  if (!(maxext > 0.0)) maxext = 1.0;
  const double fine0 = maxext / 1000.0;
  if (std::isfinite(cutoff)) {
    const double target = 0.5 * cutoff;
    int shift = 0;
    double fine = fine0;
    if (target >= fine0) {
      shift = (int)std::floor(std::log2(target / fine0));
      shift = std::min(std::max(shift, 0), 7);
      fine = target / std::ldexp(1.0, shift);
    }
    L.fine = fine;
    L.shift = shift;
  } else {
    L.fine = fine0;
    L.shift = 0;
  }
  L.coarse = L.fine * std::ldexp(1.0, L.shift);
  for (int d = 0; d < 3; ++d) {
    L.origin[d] = box[d] - 0.5 * L.fine;
    int64_t fd = (int64_t)std::floor(ext[d] / L.fine) + 2;
    L.fdims[d] = (int)std::min<int64_t>(fd, kFineMax);
    L.cdims[d] = (int)ceil_div(L.fdims[d], (int64_t)1 << L.shift);
  }
  return L;
}

void ensure_solver(Ctx* c, int m) {
  if (c->V && c->krylov_m >= m) return;
  dfree(c->V);
  // m + 1 basis vectors, rounded up to whole blocks of the dot-product
  // kernels' column loop (they read the extra columns, zero, unguarded)
  const int64_t cols = round_up(m + 1, kKrylovColPad);
  c->V = dalloc<double>(cols * c->mpad);
  RBF_HIP(hipMemsetAsync(c->V, 0, sizeof(double) * (size_t)(cols * c->mpad), temp_stream()));
  c->krylov_m = m;
  if (!c->w) {
    c->w = dalloc<double>(c->mpad);
    c->r = dalloc<double>(c->mpad);
    c->csol = dalloc<double>(c->mpad);
    c->bsort = dalloc<double>(c->mpad);
    RBF_HIP(hipMemsetAsync(c->w, 0, sizeof(double) * c->mpad, temp_stream()));
    RBF_HIP(hipMemsetAsync(c->r, 0, sizeof(double) * c->mpad, temp_stream()));
    RBF_HIP(hipMemsetAsync(c->csol, 0, sizeof(double) * c->mpad, temp_stream()));
    RBF_HIP(hipMemsetAsync(c->bsort, 0, sizeof(double) * c->mpad, temp_stream()));
    c->state = dalloc<char>((int64_t)gm_state_bytes());
    RBF_HIP(hipMemsetAsync(c->state, 0, gm_state_bytes(), temp_stream()));
  } else {
    RBF_HIP(hipMemsetAsync(c->w, 0, sizeof(double) * c->mpad, temp_stream()));
  }
  // the basis and w are all zero bits: 0 read as float32 or as float64
  c->krylov_f32 = -1;
  const int64_t pc = gm_partial_count(c->m);
  if (c->partial_cap < pc) {
    dfree(c->partial);
    c->partial = dalloc<double>(pc);
    c->partial_cap = pc;
  }
}

// The basis and w are reinterpreted as float32 or float64 storage: on a
// change of type the padding entry m of every basis vector (a weight of the
// operator) must read 0 in the new element type too.
void set_basis_type(Ctx* c, bool f32, hipStream_t s) {
  if (c->krylov_f32 != (int)f32 && c->krylov_f32 != -1) {
    fill_f64(c->V, 0.0, round_up(c->krylov_m + 1, kKrylovColPad) * c->mpad, s);
    fill_f64(c->w, 0.0, c->mpad, s);
  }
  c->krylov_f32 = (int)f32;
}

// y_sorted = A x_sorted (x_sorted has a zero at index m).
void apply_sorted(Ctx* c, const double* x, double* y, int prec, hipStream_t s, const int* skip = nullptr) {
  if (prec == RBF_FP32)
    pairsum_f32(*c, c->centres, x, false, y, s, skip);
  else
    pairsum_f64(*c, c->centres, x, false, y, s, skip);
}

}  // namespace

void set_thread_error(const std::string& msg) { t_err = msg; }
const char* thread_error() { return t_err.c_str(); }

}  // namespace rbf

using namespace rbf;

struct rbf_ctx : rbf::Ctx {};

extern "C" {

int rbf_default_solve_opts(rbf_solve_opts* o) {
  if (!o) return fail(nullptr, RBF_EINVAL, "opts is NULL");
  o->tol = 1e-8;
  o->restart = 30;
  o->max_outer = 1000;
  o->max_iters = 30000;
  o->mode = RBF_SOLVE_IR_FP32;
  o->precond = RBF_PRECOND_NONE;
  o->basis = RBF_FP32;
  o->graph = 1;
  return RBF_OK;
}

int rbf_setup(const double* points, const double* normals, int64_t n, double off_surface_eps, double sigma,
              double cutoff, void* stream, rbf_ctx** out) {
  TempStream temp_scope((hipStream_t)stream);
  if (!out) return fail(nullptr, RBF_EINVAL, "out is NULL");
  *out = nullptr;
  if (n <= 0) return fail(nullptr, RBF_EINVAL, "n must be positive");
  if (n > ((int64_t)1 << 29)) return fail(nullptr, RBF_EINVAL, "n too large (3n must fit 31-bit indices)");
  if (!(off_surface_eps > 0.0) || !std::isfinite(off_surface_eps))
    return fail(nullptr, RBF_EINVAL, "off_surface_eps must be finite and > 0");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(nullptr, RBF_EINVAL, "sigma must be finite and > 0");
  if (!(cutoff > 0.0)) return fail(nullptr, RBF_EINVAL, "cutoff must be > 0 (or +INFINITY)");
  int dev = 0;
  int st = check_device(nullptr, &dev);
  if (st != RBF_OK) return st;
  if (!is_device_ptr(points) || !is_device_ptr(normals))
    return fail(nullptr, RBF_EINVAL, "points and normals must be device pointers");
  rbf_ctx* c = new (std::nothrow) rbf_ctx();
  if (!c) return fail(nullptr, RBF_ENOMEM, "host allocation failed");
  hipStream_t s = (hipStream_t)stream;
  st = guarded(c, [&]() -> int {
    c->device = dev;
    c->n = n;
    c->m = 3 * n;
    c->mpad = round_up(c->m + 1, 256);
    c->eps = off_surface_eps;
    c->sigma = sigma;
    c->cutoff = cutoff;
    c->rc2 = std::isfinite(cutoff) ? cutoff * cutoff : INFINITY;
    c->sqrt_k = std::sqrt(1.4426950408889634 / (2.0 * sigma * sigma));
    c->inv_two_s2 = 1.0 / (2.0 * sigma * sigma);
    // 1. inputs (the flags are read back with the bounding box, one wait
    // for both; the two kernels in between only combine values elementwise,
    // so bad inputs make bad values there and nothing else)
    int* flags = talloc<int>(2);
    RBF_HIP(hipMemsetAsync(flags, 0, 2 * sizeof(int), s));
    check_inputs(points, normals, n, flags, s);
    // 2. extended set (paper order)
    c->xpaper = dalloc<double>(3 * c->m);
    build_centres(points, normals, n, off_surface_eps, c->xpaper, s);
    // 3. lattice from the bounding box
    double* box = talloc<double>(6 + 6 * 1024);
    bounding_box(c->xpaper, c->m, box, box + 6, s);
    int hf[2] = {0, 0};
    double hb[6];
    {
      PinnedSlots rb(7);   // the two flags in slot 0, the box in slots 1..6
      RBF_HIP(hipMemcpyAsync(rb.p, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
      RBF_HIP(hipMemcpyAsync(rb.p + 1, box, sizeof(hb), hipMemcpyDeviceToHost, s));
      RBF_HIP(hipStreamSynchronize(s));
      std::memcpy(hf, rb.p, sizeof(hf));
      std::memcpy(hb, rb.p + 1, sizeof(hb));
    }
    temp_free(flags);
    temp_free(box);
    if (hf[0]) return fail(c, RBF_EINVAL, "points or normals contain NaN or Inf");
    if (hf[1]) return fail(c, RBF_EINVAL, "a normal is shorter than 1e-12");
    c->lat = make_lattice(hb, cutoff);
    if (std::isfinite(cutoff)) {
      const double cells = (double)c->lat.cdims[0] * c->lat.cdims[1] * c->lat.cdims[2];
      if (cells > (double)((int64_t)1 << 28))
        return fail(c, RBF_EINVAL, "cutoff too small for the extent of the cloud (neighbour lattice too large)");
    }
    // 4. Hilbert order
    c->perm = dalloc<uint32_t>(c->m);
    c->keys = dalloc<uint32_t>(c->m);
    sort_points(c->xpaper, c->m, c->lat, c->perm, c->keys, s);
    c->xs = dalloc<double4>(c->m + 1);
    c->xk = dalloc<double4>(c->m + 1);
    gather_sorted(c->xpaper, c->perm, c->m, c->sqrt_k, c->xs, c->xk, s);
    // 5. coarse cells
    PinnedSlots late(3);   // read after the final wait: the cell count's two parts, the inner entries
    int64_t* ncell_parts = late.p;
    ncell_parts[0] = ncell_parts[1] = 0;
    if (std::isfinite(cutoff)) {
      build_cells(c->keys, c->xs, c->m, c->lat, &c->cell_start, &c->cell_count, &c->cell_map, &c->cell_xyz,
                  ncell_parts, s);
      c->cell_sat = build_cell_sat(*c, s);
    }
    // 6. the centres as targets, with their source lists
    TargetSet& ts = c->centres;
    ts.dense = !std::isfinite(cutoff);
    centre_targets(*c, ts, s);
    build_lists(*c, ts, s, late.p + 2);
    // 7. work vectors
    c->vin = dalloc<double>(c->mpad);
    c->vout = dalloc<double>(c->mpad);
    RBF_HIP(hipMemsetAsync(c->vin, 0, sizeof(double) * c->mpad, s));
    RBF_HIP(hipMemsetAsync(c->vout, 0, sizeof(double) * c->mpad, s));
    RBF_HIP(hipStreamSynchronize(s));
    c->n_cells = ncell_parts[0] + ncell_parts[1];
    ts.inner_entries = late.p[2];
    return RBF_OK;
  });
  if (st != RBF_OK) {
    t_err = c->err;
    free_ctx(c);
    delete c;
    return st;
  }
  *out = c;
  return RBF_OK;
}

int rbf_centres(rbf_ctx* c, double* centres, double* values, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  if ((centres && !is_device_ptr(centres)) || (values && !is_device_ptr(values)))
    return fail(c, RBF_EINVAL, "outputs must be device pointers");
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    if (centres)
      RBF_HIP(hipMemcpyAsync(centres, c->xpaper, sizeof(double) * 3 * c->m, hipMemcpyDeviceToDevice, s));
    if (values) {
      fill_f64(values, 0.0, c->n, s);
      fill_f64(values + c->n, c->eps, c->n, s);
      fill_f64(values + 2 * c->n, -c->eps, c->n, s);
    }
    return RBF_OK;
  });
}

int rbf_matvec(rbf_ctx* c, const double* x, double* y, int prec, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  if (prec != RBF_FP32 && prec != RBF_FP64) return fail(c, RBF_EINVAL, "prec must be RBF_FP32 or RBF_FP64");
  if (!is_device_ptr(x) || !is_device_ptr(y)) return fail(c, RBF_EINVAL, "x and y must be device pointers");
  if (x == y) return fail(c, RBF_EINVAL, "x and y must not overlap");
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    gather_to_sorted(x, c->perm, c->m, c->vin, s);
    apply_sorted(c, c->vin, c->vout, prec, s);
    scatter_from_sorted(c->vout, c->perm, c->m, y, s);
    return RBF_OK;
  });
}

int rbf_solve(rbf_ctx* c, const double* b, const double* x0, double* cout, const rbf_solve_opts* opts_in,
              rbf_solve_info* info, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  rbf_solve_opts o;
  rbf_default_solve_opts(&o);
  if (opts_in) o = *opts_in;
  if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) return fail(c, RBF_EINVAL, "tol must be finite and >= 0");
  if (o.restart < 1 || o.restart > gm_max_restart()) return fail(c, RBF_EINVAL, "restart must be in 1..64");
  if (o.max_outer < 1 || o.max_iters < 0) return fail(c, RBF_EINVAL, "max_outer >= 1 and max_iters >= 0 required");
  if (o.mode != RBF_SOLVE_PLAIN_FP64 && o.mode != RBF_SOLVE_IR_FP32) return fail(c, RBF_EINVAL, "unknown mode");
  if (o.precond != RBF_PRECOND_NONE && o.precond != RBF_PRECOND_SCHWARZ)
    return fail(c, RBF_EINVAL, "unknown preconditioner");
  if (o.basis != RBF_FP32 && o.basis != RBF_FP64) return fail(c, RBF_EINVAL, "basis must be RBF_FP32 or RBF_FP64");
  if (o.graph != 0 && o.graph != 1) return fail(c, RBF_EINVAL, "graph must be 0 or 1");
  if (o.precond == RBF_PRECOND_SCHWARZ && !c->schwarz)
    return fail(c, RBF_EINVAL, "no Schwarz preconditioner on this context (rbf_schwarz_setup)");
  if ((b && !is_device_ptr(b)) || (x0 && !is_device_ptr(x0)) || !is_device_ptr(cout))
    return fail(c, RBF_EINVAL, "b, x0 and c must be device pointers");
  const int prec = o.mode == RBF_SOLVE_IR_FP32 ? RBF_FP32 : RBF_FP64;
  int result = guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    ensure_solver(c, o.restart);
    const int64_t m = c->m;
    const int64_t ldv = c->mpad;
    // b and x0 in sorted order
    if (b) {
      gather_to_sorted(b, c->perm, m, c->bsort, s);
    } else {
      // values 0 / +eps / -eps of the paper order, written in sorted order
      rhs_sorted(c->perm, m, c->n, c->eps, c->bsort, s);
    }
    bool have_x = x0 != nullptr;
    if (x0)
      gather_to_sorted(x0, c->perm, m, c->csol, s);
    else
      fill_f64(c->csol, 0.0, c->mpad, s);
    // the inner solve of the refinement keeps its Krylov basis (and w) in
    // float32 unless asked otherwise, in the same allocations; the plain
    // method in float64
    const bool f32 = o.mode == RBF_SOLVE_IR_FP32 && o.basis == RBF_FP32;
    set_basis_type(c, f32, s);
    gm_start(c->bsort, nullptr, c->r, m, c->V, f32, c->partial, o.restart, 0.0, c->state, s);
    int k, done, bd;
    double bnorm, gk;
    gm_read(c->state, &k, &done, &bd, &bnorm, &gk, s);
    c->history.clear();
    c->history_ms.clear();
    const auto t_start = std::chrono::steady_clock::now();
    auto stamp = [&](double rel) {
      c->history.push_back(rel);
      c->history_ms.push_back(
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count());
    };
    int iters = 0, outer = 0, status = RBF_ENOCONV;
    double rel = 0.0;
    if (!std::isfinite(bnorm)) {
      status = RBF_EBREAKDOWN;
    } else if (bnorm == 0.0) {
      fill_f64(c->csol, 0.0, c->mpad, s);
      rel = 0.0;
      stamp(0.0);
      status = RBF_OK;
    } else {
      // without a starting guess the cycle started above (r = b) is the
      // first one: it only needs its stopping tolerance
      bool first_started = !have_x;
      if (first_started) gm_set_tol(c->state, o.tol * bnorm, s);
      bool residual_queued = false;
      for (;;) {
        double beta;
        if (first_started) {
          beta = bnorm;
          first_started = false;
        } else {
          // true residual with the float64 operator (queued already when a
          // cycle has just ended)
          const double* y = nullptr;
          if (have_x) {
            if (!residual_queued) apply_sorted(c, c->csol, c->vout, RBF_FP64, s);
            y = c->vout;
          }
          residual_queued = false;
          gm_start(c->bsort, y, c->r, m, c->V, f32, c->partial, o.restart, o.tol * bnorm, c->state, s);
          gm_read(c->state, &k, &done, &bd, &beta, &gk, s);
        }
        rel = beta / bnorm;
        stamp(rel);
        if (!std::isfinite(rel)) {
          status = RBF_EBREAKDOWN;
          break;
        }
        if (rel <= o.tol) {
          status = RBF_OK;
          break;
        }
        if (outer >= o.max_outer || iters >= o.max_iters) {
          status = RBF_ENOCONV;
          break;
        }
        const int steps = std::min<int64_t>(o.restart, (int64_t)o.max_iters - iters);
        const int* skip = gm_done_flag(c->state);
        const SchwarzData* pre = o.precond == RBF_PRECOND_SCHWARZ ? c->schwarz : nullptr;
        // the Arnoldi steps of the cycle, on stream st (launches only: no
        // allocation, copy or wait, so that they can be captured)
        auto arnoldi_steps = [&](hipStream_t st, int count) {
          for (int j = 0; j < count; ++j) {
            if (f32) {
              const float* vj = reinterpret_cast<const float*>(c->V) + (int64_t)j * ldv;
              float* w = reinterpret_cast<float*>(c->w);
              if (pre) {
                // right preconditioning: the basis is built on A M (M applied
                // to the float32 basis vector, its result rounded to float32
                // for the float32 operator)
                schwarz_apply_f32(*c, *pre, vj, pre->z32, st, skip);
                pairsum_f32(*c, c->centres, nullptr, true, w, st, skip, pre->z32);
              } else {
                pairsum_f32(*c, c->centres, nullptr, true, w, st, skip, vj);
              }
            } else {
              const double* vj = c->V + (int64_t)j * ldv;
              if (pre) {
                schwarz_apply(*c, *pre, vj, pre->z, st, skip);
                vj = pre->z;
              }
              apply_sorted(c, vj, c->w, prec, st, skip);
            }
            gm_step(c->V, ldv, c->w, f32, m, j, c->partial, c->state, st);
          }
        };
        // Full cycles replay a captured graph of these launches.  Capturing
        // and instantiating takes the host about a millisecond, so a cycle
        // without a graph is launched directly, and the graph is captured
        // afterwards (while the device runs that cycle) only when another
        // full cycle may follow.
        const bool use_graph = o.graph && steps == o.restart && !profiling();
        std::vector<intptr_t> key;
        if (use_graph)
          key = {o.restart, f32, prec, (intptr_t)pre, (intptr_t)c->V, (intptr_t)c->w, (intptr_t)c->vin,
                 (intptr_t)c->partial, (intptr_t)c->state, (intptr_t)ldv, (intptr_t)m};
        if (use_graph && c->cycle_exec && c->cycle_key == key) {
          RBF_HIP(hipGraphLaunch(c->cycle_exec, s));
        } else {
          arnoldi_steps(s, steps);
          const bool later_full = outer + 1 < o.max_outer && (int64_t)o.max_iters - iters - steps >= o.restart;
          if (use_graph && later_full) {
            drop_cycle_graph(c);
            if (!c->capture_stream) RBF_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            RBF_HIP(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeRelaxed));
            try {
              arnoldi_steps(c->capture_stream, steps);
            } catch (...) {
              (void)hipStreamEndCapture(c->capture_stream, &g);
              if (g) (void)hipGraphDestroy(g);
              throw;
            }
            RBF_HIP(hipStreamEndCapture(c->capture_stream, &g));
            hipGraphExec_t ex = nullptr;
            const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            RBF_HIP(e);
            c->cycle_exec = ex;
            c->cycle_key = key;
          }
        }
        if (pre) {
          // c += M (V y)
          fill_f64(pre->t, 0.0, c->mpad, s);
          gm_finish(c->V, ldv, f32, pre->t, m, c->state, s);
          schwarz_apply(*c, *pre, pre->t, pre->z, s);
          vec_add(c->csol, pre->z, m, s);
        } else {
          gm_finish(c->V, ldv, f32, c->csol, m, c->state, s);
        }
        // the next true residual goes into the queue before the host waits
        // for the cycle's state, so that the device is not idle meanwhile
        apply_sorted(c, c->csol, c->vout, RBF_FP64, s);
        residual_queued = true;
        gm_read(c->state, &k, &done, &bd, &beta, &gk, s);
        iters += k;
        ++outer;
        have_x = true;
        if (bd) {
          status = RBF_EBREAKDOWN;
          // the true residual of the current iterate is still reported
          gm_start(c->bsort, c->vout, c->r, m, c->V, f32, c->partial, o.restart, 0.0, c->state, s);
          gm_read(c->state, &k, &done, &bd, &beta, &gk, s);
          rel = beta / bnorm;
          stamp(rel);
          break;
        }
        if (k == 0 && steps > 0) {
          // no progress possible (degenerate Krylov space)
          status = RBF_ENOCONV;
          break;
        }
      }
    }
    scatter_from_sorted(c->csol, c->perm, m, cout, s);
    RBF_HIP(hipStreamSynchronize(s));
    if (info) {
      info->iters = iters;
      info->outer = outer;
      info->rel_resid = rel;
      info->status = status;
      info->n_history = (int)c->history.size();
      info->history = c->history.data();
      info->history_ms = c->history_ms.data();
    }
    if (status == RBF_ENOCONV) c->err = "solve stopped at its iteration limit";
    if (status == RBF_EBREAKDOWN) c->err = "non-finite value in the solve";
    return status;
  });
  if (result == RBF_ENOCONV || result == RBF_EBREAKDOWN) t_err = c->err;
  return result;
}

static int check_grid(rbf_ctx* c, const rbf_grid* g) {
  if (!g) return fail(c, RBF_EINVAL, "grid is NULL");
  for (int d = 0; d < 3; ++d) {
    if (g->dims[d] <= 0) return fail(c, RBF_EINVAL, "grid dims must be positive");
    if (!std::isfinite(g->origin[d]) || !std::isfinite(g->h[d]) || g->h[d] < 0.0)
      return fail(c, RBF_EINVAL, "grid origin/h must be finite, h >= 0");
  }
  const double total = (double)g->dims[0] * (double)g->dims[1] * (double)g->dims[2];
  if (total > 4.0e9) return fail(c, RBF_EINVAL, "grid too large");
  return RBF_OK;
}

int rbf_eval_grid(rbf_ctx* c, const double* cw, const rbf_grid* grid, void* out, int prec, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  int st = check_grid(c, grid);
  if (st != RBF_OK) return st;
  if (prec != RBF_FP32 && prec != RBF_FP64) return fail(c, RBF_EINVAL, "prec must be RBF_FP32 or RBF_FP64");
  if (!is_device_ptr(cw) || !is_device_ptr(out)) return fail(c, RBF_EINVAL, "c and out must be device pointers");
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    const int64_t total = grid->dims[0] * grid->dims[1] * grid->dims[2];
    gather_to_sorted(cw, c->perm, c->m, c->vin, s);
    if (prec == RBF_FP32)
      fill_f32(static_cast<float*>(out), 0.0f, total, s);
    else
      fill_f64(static_cast<double*>(out), 0.0, total, s);
    if (prec == RBF_FP32 && brick_sum_applies(*c, *grid)) {
      // float32 with a cutoff: tiles of bricks walk their candidate sources
      // directly
      int64_t* ws = talloc<int64_t>(support_tiles_ws_elems(*grid));
      const int64_t *tiles = nullptr, *masks = nullptr;
      const int64_t nt = support_tiles(*c, *grid, ws, &tiles, &masks, s);
      // (timed like the pair kernels; it counts no pairs: the counts of a
      // grid come from rbf_count_grid_pairs)
      ProfScope ps(RBF_FP32, 1, 0, 0, s);
      brick_sum_tiles(*c, *grid, tiles, masks, nt, c->vin, static_cast<float*>(out), nullptr, nullptr, s,
                      ps.start(), ps.stop());
      ps.done();
      RBF_HIP(hipStreamSynchronize(s));
      temp_free(ws);
      return RBF_OK;
    }
    TargetSet ts;
    grid_targets(*c, *grid, ts, s);
    if (ts.n_groups > 0) {
      if (prec == RBF_FP32)
        pairsum_f32(*c, ts, c->vin, true, out, s);
      else
        pairsum_f64(*c, ts, c->vin, false, out, s);
    }
    RBF_HIP(hipStreamSynchronize(s));
    free_targets(ts);
    return RBF_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free float32 grid evaluation (rbf_eval_grid_noalloc).  Its only
// scratch memory (the brick marks, their scan and the list of bricks with a
// centre in reach) lives in `scratch`, a fixed array in device memory: each
// device the library runs on holds its own copy until the process ends.  In
// host code the array's name is not a device address; its address on a
// device comes from hipGetSymbolAddress, looked up once per device with that
// device current, and only that address is handed to kernels.
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kNoAllocMaxBricks = int64_t(1) << 21;           // bricks of 4 x 2 x 2 nodes
constexpr int64_t kNoAllocScratch = 3 * kNoAllocMaxBricks + 8192;  // int64 entries: 48 MiB + 64 KiB
static __device__ __align__(256) int64_t scratch[kNoAllocScratch];

int64_t* scratch_address(int dev) {
  static std::mutex mu;
  static std::map<int, int64_t*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  int64_t* p = nullptr;
  RBF_HIP(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error{RBF_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array"};
  addr.emplace(dev, p);
  return p;
}

}  // namespace

extern "C" {

int rbf_eval_grid_noalloc(rbf_ctx* c, const double* cw, const rbf_grid* grid, float* out, void* stream) {
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  int st = check_grid(c, grid);
  if (st != RBF_OK) return st;
  if (!is_device_ptr(cw) || !is_device_ptr(out)) return fail(c, RBF_EINVAL, "c and out must be device pointers");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
    return fail(c, RBF_EINVAL, "the context's device must be the current device");
  if (!brick_sum_applies(*c, *grid))
    return fail(c, RBF_EINVAL,
                "rbf_eval_grid_noalloc sums float32 grids brick by brick: it needs a cutoff and a grid spacing "
                "fine against sigma (rbf_eval_grid handles the other grids)");
  const GridDesc gd = grid_desc(*grid);
  const int64_t nbricks = gd.nb[0] * gd.nb[1] * gd.nb[2];
  if (nbricks > kNoAllocMaxBricks || support_tiles_ws_elems(*grid) > kNoAllocScratch)
    return fail(c, RBF_EINVAL,
                "grid of " + std::to_string(nbricks) + " bricks of 4 x 2 x 2 nodes: rbf_eval_grid_noalloc holds at "
                "most " + std::to_string(kNoAllocMaxBricks) + " (use rbf_eval_grid)");
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    int64_t* ws = scratch_address(dev);
    const int64_t total = grid->dims[0] * grid->dims[1] * grid->dims[2];
    gather_to_sorted(cw, c->perm, c->m, c->vin, s);
    fill_f32(out, 0.0f, total, s);
    const int64_t *tiles = nullptr, *masks = nullptr;
    const int64_t nt = support_tiles(*c, *grid, ws, &tiles, &masks, s, /*pinned=*/false);
    brick_sum_tiles(*c, *grid, tiles, masks, nt, c->vin, out, nullptr, nullptr, s);
    RBF_HIP(hipStreamSynchronize(s));
    return RBF_OK;
  });
}

int rbf_count_grid_pairs(rbf_ctx* c, const rbf_grid* grid, int64_t* useful, int64_t* examined, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  int st = check_grid(c, grid);
  if (st != RBF_OK) return st;
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    TargetSet ts;
    grid_targets(*c, *grid, ts, s);
    if (useful) *useful = ts.useful;
    if (examined) *examined = ts.list_entries * kGroup;
    free_targets(ts);
    return RBF_OK;
  });
}

int rbf_eval_points(rbf_ctx* c, const double* cw, const double* pts, int64_t npts, double* out, int prec,
                    void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  if (npts < 0) return fail(c, RBF_EINVAL, "m must be >= 0");
  if (prec != RBF_FP32 && prec != RBF_FP64) return fail(c, RBF_EINVAL, "prec must be RBF_FP32 or RBF_FP64");
  if (npts == 0) return RBF_OK;
  if (npts > ((int64_t)1 << 31) - 2) return fail(c, RBF_EINVAL, "too many points");
  if (!is_device_ptr(cw) || !is_device_ptr(pts) || !is_device_ptr(out))
    return fail(c, RBF_EINVAL, "c, pts and out must be device pointers");
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    gather_to_sorted(cw, c->perm, c->m, c->vin, s);
    TargetSet ts;
    point_targets(*c, pts, npts, ts, s);
    if (prec == RBF_FP32)
      pairsum_f32(*c, ts, c->vin, false, out, s);
    else
      pairsum_f64(*c, ts, c->vin, false, out, s);
    RBF_HIP(hipStreamSynchronize(s));
    free_targets(ts);
    return RBF_OK;
  });
}

int rbf_density(rbf_ctx* c, const double* samples, int64_t ns, rbf_density_info* out, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  if (!out) return fail(c, RBF_EINVAL, "out is NULL");
  if (ns < 0) return fail(c, RBF_EINVAL, "n_samples must be >= 0");
  if (samples && ns > 0 && !is_device_ptr(samples)) return fail(c, RBF_EINVAL, "samples must be a device pointer");
  return guarded(c, [&]() -> int {
    double q, hmax, hfill;
    density_measures(c->xpaper, c->n, samples, samples ? ns : 0, &q, &hmax, &hfill, (hipStream_t)stream);
    out->q = q;
    out->h_max = hmax;
    out->h_fill = hfill;
    // eq. hmax stands in for the fill distance when no domain sample is given
    out->h = std::isnan(hfill) ? std::sqrt(2.0) * hmax : hfill;
    out->sigma_sep = 2.0 * q;                    // eq. h1
    out->sigma_fill = std::sqrt(2.0) * out->h;   // eq. h2
    return RBF_OK;
  });
}

int rbf_arnoldi(rbf_ctx* c, const double* v0, int m, int op_prec, int basis, double* V, double* H, int* steps,
                void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  if (m < 1 || m > gm_max_restart()) return fail(c, RBF_EINVAL, "m must be in 1..64");
  if (op_prec != RBF_FP32 && op_prec != RBF_FP64) return fail(c, RBF_EINVAL, "op_prec must be RBF_FP32 or RBF_FP64");
  if (basis != RBF_FP32 && basis != RBF_FP64) return fail(c, RBF_EINVAL, "basis must be RBF_FP32 or RBF_FP64");
  if (!H || !steps) return fail(c, RBF_EINVAL, "H and steps must not be NULL (host)");
  if (is_device_ptr(H)) return fail(c, RBF_EINVAL, "H must be a host array");
  if (!is_device_ptr(v0) || !is_device_ptr(V)) return fail(c, RBF_EINVAL, "v0 and V must be device pointers");
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    ensure_solver(c, m);
    const int64_t n = c->m, ldv = c->mpad;
    const bool f32 = basis == RBF_FP32;
    set_basis_type(c, f32, s);
    gather_to_sorted(v0, c->perm, n, c->bsort, s);
    // v_0 = v0 / |v0|, no stopping tolerance
    gm_start(c->bsort, nullptr, c->r, n, c->V, f32, c->partial, m, 0.0, c->state, s);
    const int* skip = gm_done_flag(c->state);
    for (int j = 0; j < m; ++j) {
      if (f32)
        pairsum_f32(*c, c->centres, nullptr, true, c->w, s, skip, reinterpret_cast<const float*>(c->V) + j * ldv);
      else if (op_prec == RBF_FP32)
        pairsum_f32(*c, c->centres, c->V + j * ldv, false, c->w, s, skip);
      else
        pairsum_f64(*c, c->centres, c->V + j * ldv, false, c->w, s, skip);
      gm_step(c->V, ldv, c->w, f32, n, j, c->partial, c->state, s);
    }
    int bd = 0;
    const int k = gm_read_hessenberg(c->state, m, H, &bd, s);
    *steps = k;
    // basis vectors in paper order (float64); the last one exists only when
    // every step ran to the end
    const int rows = k == m && !bd ? m + 1 : k;
    fill_f64(V, 0.0, (int64_t)(m + 1) * n, s);
    for (int r = 0; r < rows; ++r) {
      const double* col = c->V + r * ldv;
      if (f32) {
        to_f64(reinterpret_cast<const float*>(c->V) + r * ldv, c->vin, n, s);
        col = c->vin;
      }
      scatter_from_sorted(col, c->perm, n, V + (int64_t)r * n, s);
    }
    RBF_HIP(hipStreamSynchronize(s));
    if (bd) return fail(c, RBF_EBREAKDOWN, "non-finite value in the Arnoldi process");
    return RBF_OK;
  });
}

int rbf_default_schwarz_opts(rbf_schwarz_opts* o) {
  if (!o) return fail(nullptr, RBF_EINVAL, "opts is NULL");
  o->max_block = kSchwarzDefaultBlock;
  o->overlap_pct = 10;
  o->restricted = 0;
  o->min_block = 0;
  o->shift = 0.3;
  o->tune = 1;
  o->half = 0;
  return RBF_OK;
}

int rbf_schwarz_setup(rbf_ctx* c, const rbf_schwarz_opts* opts_in, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  rbf_schwarz_opts o;
  rbf_default_schwarz_opts(&o);
  if (opts_in) o = *opts_in;
  if (o.max_block < 3 || o.max_block > kSchwarzMaxBlock)
    return fail(c, RBF_EINVAL, "max_block must be in 3..1024");
  if (o.min_block < 0 || o.min_block > o.max_block) return fail(c, RBF_EINVAL, "min_block must be in 0..max_block");
  if (o.tune != 0 && o.tune != 1) return fail(c, RBF_EINVAL, "tune must be 0 or 1");
  if (o.overlap_pct < 0 || o.overlap_pct > 100) return fail(c, RBF_EINVAL, "overlap_pct must be in 0..100");
  if (o.restricted != 0 && o.restricted != 1) return fail(c, RBF_EINVAL, "restricted must be 0 or 1");
  if (o.half != 0 && o.half != 1) return fail(c, RBF_EINVAL, "half must be 0 or 1");
  if (!(o.shift >= 0.0) || !std::isfinite(o.shift)) return fail(c, RBF_EINVAL, "shift must be finite and >= 0");
  if (3 + schwarz_overlap_count(3, o.overlap_pct) > o.max_block)
    return fail(c, RBF_EINVAL, "max_block too small for one point and its overlap");
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    drop_cycle_graph(c);        // it may hold the old preconditioner's launches
    free_schwarz(c->schwarz);   // stream-ordered release: queued work on this stream finishes first
    c->schwarz = nullptr;
    c->schwarz =
        schwarz_setup(*c, o.max_block, o.overlap_pct, o.restricted, o.min_block, o.shift, o.tune, o.half != 0, s);
    RBF_HIP(hipStreamSynchronize(s));
    return RBF_OK;
  });
}

int rbf_schwarz_apply(rbf_ctx* c, const double* r, double* z, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  if (!c->schwarz) return fail(c, RBF_EINVAL, "no Schwarz preconditioner on this context (rbf_schwarz_setup)");
  if (!is_device_ptr(r) || !is_device_ptr(z)) return fail(c, RBF_EINVAL, "r and z must be device pointers");
  if (r == z) return fail(c, RBF_EINVAL, "r and z must not overlap");
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    gather_to_sorted(r, c->perm, c->m, c->vin, s);
    schwarz_apply(*c, *c->schwarz, c->vin, c->vout, s);
    scatter_from_sorted(c->vout, c->perm, c->m, z, s);
    return RBF_OK;
  });
}

int rbf_schwarz_get_info(const rbf_ctx* c, rbf_schwarz_info* out) {
  if (!c || !out) return fail(nullptr, RBF_EINVAL, "ctx and info must not be NULL");
  if (!c->schwarz) return fail(const_cast<rbf_ctx*>(c), RBF_EINVAL, "no Schwarz preconditioner on this context");
  const SchwarzData& d = *c->schwarz;
  out->n_sub = d.nsub;
  out->n_members = d.nmem;
  int64_t maxn = 0, minn = d.nsub > 0 ? INT64_MAX : 0;
  for (int64_t i = 0; i < d.nsub; ++i) {
    maxn = std::max(maxn, d.h_mem_off[i + 1] - d.h_mem_off[i]);
    minn = std::min(minn, d.h_mem_off[i + 1] - d.h_mem_off[i]);
  }
  out->max_members = maxn;
  out->min_members = minn;
  out->inverse_bytes = d.w_total * (int64_t)(d.half ? sizeof(_Float16) : sizeof(float));
  out->retries = d.retries;
  out->max_shift = d.max_shift;
  out->apply_threads = d.apply_threads;
  out->apply_blocks = d.apply_blocks;
  out->factor_ms = d.factor_ms;
  return RBF_OK;
}

int rbf_schwarz_subdomains(const rbf_ctx* c, int64_t* offsets, int32_t* n_core, int64_t* members) {
  if (!c || !offsets || !n_core || !members) return fail(nullptr, RBF_EINVAL, "NULL argument");
  if (!c->schwarz) return fail(const_cast<rbf_ctx*>(c), RBF_EINVAL, "no Schwarz preconditioner on this context");
  const SchwarzData& d = *c->schwarz;
  for (int64_t i = 0; i <= d.nsub; ++i) offsets[i] = d.h_mem_off[i];
  for (int64_t i = 0; i < d.nsub; ++i) n_core[i] = d.h_ncore[i];
  for (int64_t e = 0; e < d.nmem; ++e) members[e] = d.h_mem_paper[e];
  return RBF_OK;
}

int rbf_net_set(rbf_ctx* c, const float* params, const double centre[3], double scale, double tau, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  if (!params || !centre) return fail(c, RBF_EINVAL, "params and centre must not be NULL (host arrays)");
  if (is_device_ptr(params)) return fail(c, RBF_EINVAL, "params must be a host array");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(centre[d])) return fail(c, RBF_EINVAL, "centre must be finite");
  if (!(scale > 0.0) || !std::isfinite(scale) || !(tau > 0.0) || !std::isfinite(tau))
    return fail(c, RBF_EINVAL, "scale and tau must be finite and > 0");
  for (int i = 0; i < RBF_NET_PARAMS; ++i)
    if (!std::isfinite(params[i])) return fail(c, RBF_EINVAL, "params must be finite");
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    free_net(c->net);
    c->net = nullptr;
    c->net = net_create(params, centre, scale, tau, s);
    RBF_HIP(hipStreamSynchronize(s));
    return RBF_OK;
  });
}

int rbf_net_get(rbf_ctx* c, float* params, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c || !params) return fail(c, RBF_EINVAL, "ctx and params must not be NULL");
  if (!c->net) return fail(c, RBF_EINVAL, "no network on this context (rbf_net_set)");
  if (is_device_ptr(params)) return fail(c, RBF_EINVAL, "params must be a host array");
  return guarded(c, [&]() -> int {
    net_get(*c->net, params, (hipStream_t)stream);
    return RBF_OK;
  });
}

int rbf_net_forward(rbf_ctx* c, const double* x, int64_t n, float* y, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  if (!c->net) return fail(c, RBF_EINVAL, "no network on this context (rbf_net_set)");
  if (n < 0) return fail(c, RBF_EINVAL, "n must be >= 0");
  if (n > 0 && (!is_device_ptr(x) || !is_device_ptr(y))) return fail(c, RBF_EINVAL, "x and y must be device pointers");
  return guarded(c, [&]() -> int {
    net_forward(*c->net, x, n, y, (hipStream_t)stream);
    return RBF_OK;
  });
}

int rbf_net_gradient(rbf_ctx* c, const double* x, const double* f, int64_t n, float* grad, double* loss,
                     void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  if (!c->net) return fail(c, RBF_EINVAL, "no network on this context (rbf_net_set)");
  if (n <= 0) return fail(c, RBF_EINVAL, "n must be > 0");
  if (!is_device_ptr(x) || !is_device_ptr(f) || !is_device_ptr(grad))
    return fail(c, RBF_EINVAL, "x, f and grad must be device pointers");
  return guarded(c, [&]() -> int {
    const double L = net_step(*c->net, x, f, n, grad, false, 0.0, (hipStream_t)stream);
    if (loss) *loss = L;
    return RBF_OK;
  });
}

int rbf_net_train(rbf_ctx* c, const double* x, const double* f, int64_t n, int batch, int epochs, double lr,
                  double* loss, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  if (!c->net) return fail(c, RBF_EINVAL, "no network on this context (rbf_net_set)");
  if (n <= 0 || batch <= 0 || epochs < 0) return fail(c, RBF_EINVAL, "n > 0, batch > 0 and epochs >= 0 required");
  if (!(lr > 0.0) || !std::isfinite(lr)) return fail(c, RBF_EINVAL, "lr must be finite and > 0");
  if (!is_device_ptr(x) || !is_device_ptr(f)) return fail(c, RBF_EINVAL, "x and f must be device pointers");
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    double sum = 0.0;
    int64_t cnt = 0;
    for (int e = 0; e < epochs; ++e) {
      sum = 0.0;
      cnt = 0;
      for (int64_t b0 = 0; b0 < n; b0 += batch) {
        const int64_t B = std::min<int64_t>(batch, n - b0);
        sum += B * net_step(*c->net, x + 3 * b0, f + b0, B, nullptr, true, lr, s);
        cnt += B;
      }
    }
    if (loss) *loss = cnt > 0 ? sum / (double)cnt : 0.0;
    return RBF_OK;
  });
}

int rbf_eval_grid_culled(rbf_ctx* c, const double* cw, const rbf_grid* grid, float* out, double e_val,
                         rbf_cull_stats* stats, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!c) return fail(nullptr, RBF_EINVAL, "ctx is NULL");
  int st = check_grid(c, grid);
  if (st != RBF_OK) return st;
  if (!c->net) return fail(c, RBF_EINVAL, "no network on this context (rbf_net_set)");
  if (!(e_val >= 0.0) || !std::isfinite(e_val)) return fail(c, RBF_EINVAL, "e_val must be finite and >= 0");
  if (!is_device_ptr(cw) || !is_device_ptr(out)) return fail(c, RBF_EINVAL, "c and out must be device pointers");
  return guarded(c, [&]() -> int {
    hipStream_t s = (hipStream_t)stream;
    gather_to_sorted(cw, c->perm, c->m, c->vin, s);
    NetCullStats ns;
    net_eval_grid_culled(*c, *c->net, c->vin, *grid, out, e_val, 3, &ns, s);
    RBF_HIP(hipStreamSynchronize(s));
    if (stats) {
      stats->support_bricks = ns.support_bricks;
      stats->kept_bricks = ns.kept_bricks;
      stats->useful_pairs = ns.useful_pairs;
      stats->examined_pairs = ns.examined_pairs;
    }
    return RBF_OK;
  });
}

int rbf_get_stats(const rbf_ctx* c, rbf_stats* st) {
  if (!c || !st) return fail(nullptr, RBF_EINVAL, "ctx and stats must not be NULL");
  st->n_points = c->n;
  st->n_centres = c->m;
  st->n_groups = c->centres.n_groups;
  st->list_entries = c->centres.list_entries;
  st->useful_pairs = c->centres.useful;
  st->examined_pairs = c->centres.list_entries * kGroup;
  st->n_cells = c->n_cells;
  st->cell_size = c->lat.coarse;
  st->sigma = c->sigma;
  st->cutoff = c->cutoff;
  st->eps = c->eps;
  st->inner_entries = c->centres.inner_entries;
  return RBF_OK;
}

int rbf_profile_begin(void) {
  return guarded(nullptr, []() -> int { return profile_begin(); });
}

int rbf_profile_end(rbf_profile* out) {
  return guarded(nullptr, [&]() -> int { return profile_end(out); });
}

int rbf_measure_rates(rbf_rates* out, void* stream) {
  TempStream temp_scope((hipStream_t)stream);
  if (!out) return fail(nullptr, RBF_EINVAL, "out is NULL");
  return guarded(nullptr, [&]() -> int {
    measure_rates(out, (hipStream_t)stream);
    return RBF_OK;
  });
}

void rbf_destroy(rbf_ctx* c) {
  if (!c) return;
  free_ctx(c);
  delete c;
}

const char* rbf_last_error(const rbf_ctx* c) {
  if (c) return c->err.empty() ? "no error" : c->err.c_str();
  return thread_error();
}

}  // extern "C"
