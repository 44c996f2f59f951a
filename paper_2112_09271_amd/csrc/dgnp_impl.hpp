// Internal declarations of the dgnp library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dgnp.h"

namespace dgnp {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

#define DGNP_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::dgnp::Error(DGNP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define DGNP_REQUIRE(cond, code, msg)                            \
  do {                                                           \
    if (!(cond)) throw ::dgnp::Error((code), std::string(msg));  \
  } while (0)

// Device allocator of a context: the caller's hook (dgnp_options.alloc /
// free_ / alloc_ctx), or hipMalloc / hipFree when both are null.
struct DevAllocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free_)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
// The allocator that DevBuf::alloc uses on this thread: set for the duration
// of an ABI call on a context that has a hook (null: hipMalloc).  Buffers
// allocated on other threads (host helper threads) use hipMalloc.
extern thread_local const DevAllocator* t_dev_alloc;
struct AllocScope {
  const DevAllocator* prev;
  explicit AllocScope(const DevAllocator& a) : prev(t_dev_alloc) { t_dev_alloc = a.alloc ? &a : nullptr; }
  ~AllocScope() { t_dev_alloc = prev; }
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;
};

// Owning device buffer; it frees through the allocator that allocated it.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;    // elements in use
  size_t cap = 0;  // elements allocated
  DevAllocator al;  // hook of the allocation (null: hipMalloc)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), cap(o.cap), al(o.al) {
    o.p = nullptr;
    o.n = o.cap = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      cap = o.cap;
      al = o.al;
      o.p = nullptr;
      o.n = o.cap = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  // exactly count elements (a new allocation unless the size is unchanged)
  void alloc(size_t count) {
    if (count == n && p) return;
    release();
    if (count == 0) return;
    const DevAllocator* a = t_dev_alloc;
    if (a && a->alloc) {
      p = static_cast<T*>(a->alloc(count * sizeof(T), a->ctx));
      if (!p) throw Error(DGNP_E_ALLOC, "allocator hook returned NULL for " + std::to_string(count * sizeof(T)) + " bytes");
      al = *a;
    } else {
      if (hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)) != hipSuccess) {
        p = nullptr;
        throw Error(DGNP_E_ALLOC, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
      }
      al = DevAllocator{};
    }
    n = cap = count;
  }
  // count elements, keeping the allocation when it is large enough (arrays
  // whose length moves a little between set-ups are not reallocated)
  void fit(size_t count) {
    if (p && count <= cap) {
      n = count;
      return;
    }
    alloc(count);
  }
  void release() {
    if (p) {
      if (al.free_) {
        // as hipFree: no kernel may still use the memory when the hook gets it back
        (void)hipDeviceSynchronize();
        al.free_(p, al.ctx);
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    n = cap = 0;
    al = DevAllocator{};
  }
  // synchronous: the host source may be a temporary
  void upload(const T* host, size_t count, hipStream_t s) {
    alloc(count);
    if (count == 0) return;
    DGNP_HIP(hipMemcpyAsync(p, host, count * sizeof(T), hipMemcpyHostToDevice, s));
    DGNP_HIP(hipStreamSynchronize(s));
  }
  void upload(const std::vector<T>& v, hipStream_t s) { upload(v.data(), v.size(), s); }
};

// 1-D reference tables on [-1, 1]: Gauss-Lobatto nodes (p+1), Gauss points and
// weights (p+2), Lagrange values / derivatives at the Gauss points and at the
// two end points.
struct RefTables {
  int p = 0, nn = 0, nq = 0;
  std::vector<double> xn, xq, wq;
  std::vector<double> B, Dq;      // [nq][nn]
  std::vector<double> Dend[2];    // derivative of each basis function at -1 / +1
};
RefTables make_ref_tables(int p);

// Argument block shared by every DG kernel (passed by value).
struct KArgs {
  int64_t E;
  int n[3];
  double lo[3], h[3];
  double detJ;          // prod h/2
  double delta;         // interior penalty
  double Pe;
  int vel_kind;
  double vel_param[3];
  double vel_H, vel_ylo;
  double z[4], D[4], a[4], b[4];
  int c_bc[6], phi_bc[6];
  int64_t btag_off[6];  // first boundary-face index of each box face
  int64_t n_bface;
  const int* nbr;       // [E][2d]
  const double* bcq;    // [m][n_bface][nqf] boundary data at face points (f = 0: phi)
  const double* src;    // [m][E][nqv] volume sources or nullptr
  int objective_tag;    // box face of the objective
  int objective_kind;   // 0: outflow flux of species 1; 1: reaction rate on an electrode face
  // Butler-Volmer electrodes: reacting ion (1..m), its valence, exponents
  // alpha_a n / alpha_c n, dc_r / dc_k (k = 1..m-1, index k-1), and the
  // exchange-current profile in z (0: constant; 1: parabola about bv_zc with
  // half width bv_zhalf).  The per-point data sit in bcq: f = 0 the applied
  // potential, f = 1 the exchange current at the point.
  int bv_r;
  double bv_z, bv_aa, bv_ac, bv_dc[4];
  int bv_prof;
  double bv_zc, bv_zhalf;
  unsigned vin_mask;    // fields of the input vector that are read (the others count as zero)
  const void* jbase;    // M_JACP: out = jbase - (J v) rows when not null (same type as out)
};

enum Mode { M_RES = 0, M_JAC = 1, M_JACT = 2, M_DPE = 3, M_OBJG = 4, M_DATAT = 5, M_JACP = 6 };

// Launch one DG operator pass over all elements (kernels_dg.hip).
//   M_RES / M_DPE: xs = state (double), out = R or dR/dPe
//   M_JAC / M_JACT: xs = state, vin = v (same type T), out = J v / J^T v
//   M_JACP: as M_JAC, but only the potential rows of J v are formed and written (out[0, Nf))
//   M_OBJG: out = dJ/dx (out null: not formed), aux[E][4] = per-element (J,
//           dJ/dPe, dJ/dJ0, dJ/dphi_app) contributions (the last two: explicit
//           derivatives with respect to the objective face's electrode parameters)
//   M_DATAT: vin = lambda, aux[m][n_bface][nqf] = lambda^T dR/d(data at face points);
//           on electrode faces f = 0 the applied potential, f = 1 the exchange
//           current (amplitude of its profile)
void launch_dg(int dim, int p, int m, bool f32, int mode, const KArgs& A, const void* xs,
               const void* vin, void* out, double* aux, hipStream_t s);
void upload_ref_tables(const RefTables* tabs, int count);
// allocation-free objective value (kernels_dg.hip): the address of the static
// partial-sum array on the current device (looked up once per device), the
// largest element count it holds, and J(x) into J_dev (device double [1])
double* objective_scratch_init();
int64_t objective_scratch_max_elements();
void objective_noalloc(int dim, int p, int m, const KArgs& A, const double* x, double* scratch_dev, double* J_dev,
                       hipStream_t s);

}  // namespace dgnp
