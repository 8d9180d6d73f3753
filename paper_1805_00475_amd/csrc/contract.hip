// GPU contraction of a plan: upload the initial 0/1 tensors, run every
// pairwise step with a kernel chosen by its shape, read back the final
// scalar of every prime, and (tn_count) recombine by CRT.
//
// Step semantics (Sec. 2.1, Eq. 5; all shared bonds at once, Sec. 2.2):
//     C[c] = sum over z in {0,1}^s of A[z | xA << s] * B[z | xB << s]
// with xA = the C bits selected by maskA and xB those selected by maskB, in
// order. Arithmetic is per residue plane (one plane per blockIdx.z): centred
// int8 residues modulo a small modulus (<= 255), u32 residues modulo a 16-bit
// prime, or wrapping 64-bit counts, which are exact while the count fits
// (n <= 63).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "mfma.hpp"
#include "profile.hpp"
#include "launch.hpp"
#include "tune.hpp"

namespace tn {

// ------------------------------------------------------------------ kernels
// Every kernel is instantiated per element kind (EL_U32: residues modulo
// 16-bit primes, folded 64-bit sums; EL_U64: wrapping 64-bit counts; EL_I8:
// centred int8 residues modulo small moduli, exact integer sums reduced
// once at the end).

template <int E>
__device__ __forceinline__ void load_planes(const StepArgs& a, const void*& A, const void*& B, void*& C) {
    using T = typename ElemT<E>::T;
    const int g = blockIdx.z;
    A = static_cast<const T*>(a.A) + g * a.strideA;
    B = static_cast<const T*>(a.B) + g * a.strideB;
    C = static_cast<T*>(a.C) + g * a.strideC;
}

__device__ __forceinline__ ModSmall mod_small(const StepArgs& a) {
    const int g = blockIdx.z;
    return ModSmall{int32_t(a.p[g]), a.r2[g], a.r16[g], a.pinv[g]};
}

// Any shape: one thread per output entry, bit gathers by loops.
template <int E>
__global__ __launch_bounds__(256) void k_generic(StepArgs a) {
    using T = typename ElemT<E>::T;
    const void *pA, *pB;
    void* pC;
    load_planes<E>(a, pA, pB, pC);
    const T* A = static_cast<const T*>(pA);
    const T* B = static_cast<const T*>(pB);
    T* C = static_cast<T*>(pC);
    const ModP m{a.p[blockIdx.z], a.r2[blockIdx.z]};
    const ModSmall ms = mod_small(a);
    const uint64_t total = uint64_t(1) << a.rC;
    const uint64_t K = uint64_t(1) << a.s;
    for (uint64_t c = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < total;
         c += uint64_t(gridDim.x) * blockDim.x) {
        const T* ra = A + (pext64(c, a.maskA) << a.s);
        const T* rb = B + (pext64(c, a.maskB) << a.s);
        if constexpr (E == EL_U64) {
            uint64_t acc = 0;
            for (uint64_t z = 0; z < K; ++z) acc += ra[z] * rb[z];
            C[c] = acc;
        } else if constexpr (E == EL_I8) {
            int64_t acc = 0;
            for (uint64_t z = 0; z < K; ++z) acc += int32_t(ra[z]) * int32_t(rb[z]);
            C[c] = T(ms.center64(acc));
        } else {
            uint64_t acc = 0;
            uint32_t n3 = 0;
            for (uint64_t z = 0; z < K; ++z) {
                acc += uint64_t(ra[z]) * rb[z];
                if (++n3 == 3) {
                    acc = m.fold(acc);
                    n3 = 0;
                }
            }
            C[c] = m.finish(acc);
        }
    }
}

// Streaming step, small shared dimension (K = 2^LOGK <= 32): each thread
// owns one xA (256 consecutive xA per block iteration, so A is read once,
// coalesced) and NB consecutive xB of the block's xB chunk; the B slab is
// uniform across the block. Output positions split into a uniform part
// (block's xA base and xB chunk) and per-lane / per-j parts deposited once.
template <int E, int LOGK, int NB>
__global__ __launch_bounds__(256) void k_stream(StepArgs a) {
    using T = typename ElemT<E>::T;
    constexpr int K = 1 << LOGK;
    const void *pA, *pB;
    void* pC;
    load_planes<E>(a, pA, pB, pC);
    const T* A = static_cast<const T*>(pA);
    const T* B = static_cast<const T*>(pB);
    T* C = static_cast<T*>(pC);
    const ModP m{a.p[blockIdx.z], a.r2[blockIdx.z]};
    const ModSmall ms = mod_small(a);
    const uint64_t lane = threadIdx.x;
    const uint64_t laneC = pdep64(lane, a.maskA);
    uint64_t offB[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) offB[j] = pdep64(uint64_t(j), a.maskB);
    const uint64_t n_iter = (uint64_t(1) << a.fA) >> 8;
    const uint64_t n_chunk = (uint64_t(1) << a.fB) / NB;
    for (uint64_t cb = blockIdx.y; cb < n_chunk; cb += gridDim.y) {
        const uint64_t xb0 = cb * NB;
        const uint64_t baseB = pdep64(xb0, a.maskB);
        const T* rb = B + (xb0 << LOGK);
        for (uint64_t it = blockIdx.x; it < n_iter; it += gridDim.x) {
            const uint64_t xA = (it << 8) | lane;
            const uint64_t cA = pdep64(it << 8, a.maskA) | laneC | baseB;
            T av[K];
            const T* ra = A + (xA << LOGK);
#pragma unroll
            for (int z = 0; z < K; ++z) av[z] = ra[z];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                if constexpr (E == EL_U64) {
                    uint64_t acc = 0;
#pragma unroll
                    for (int z = 0; z < K; ++z) acc += av[z] * rb[j * K + z];
                    C[cA | offB[j]] = acc;
                } else if constexpr (E == EL_I8) {
                    // at most 32 products of magnitude 2^14: int32 is exact
                    int32_t acc = 0;
#pragma unroll
                    for (int z = 0; z < K; ++z) acc += int32_t(av[z]) * int32_t(rb[j * K + z]);
                    C[cA | offB[j]] = T(ms.center32(acc));
                } else {
                    uint64_t acc = 0;
#pragma unroll
                    for (int z = 0; z < K; ++z) {
                        acc += uint64_t(av[z]) * rb[j * K + z];
                        if (z % 3 == 2) acc = m.fold(acc);
                    }
                    C[cA | offB[j]] = m.finish(acc);
                }
            }
        }
    }
}

// Wide shared dimension, few outputs: one wavefront per output entry, lanes
// stride over z (coalesced rows of A and B), then a wavefront reduction.
template <int E>
__global__ __launch_bounds__(256) void k_rowdot(StepArgs a) {
    using T = typename ElemT<E>::T;
    const void *pA, *pB;
    void* pC;
    load_planes<E>(a, pA, pB, pC);
    const T* A = static_cast<const T*>(pA);
    const T* B = static_cast<const T*>(pB);
    T* C = static_cast<T*>(pC);
    const ModP m{a.p[blockIdx.z], a.r2[blockIdx.z]};
    const ModSmall ms = mod_small(a);
    const int lane = threadIdx.x & 63;
    const uint64_t wave = threadIdx.x >> 6;
    const uint64_t total = uint64_t(1) << a.rC;
    const uint64_t K = uint64_t(1) << a.s;
    for (uint64_t c = uint64_t(blockIdx.x) * 4 + wave; c < total; c += uint64_t(gridDim.x) * 4) {
        const T* ra = A + (pext64(c, a.maskA) << a.s);
        const T* rb = B + (pext64(c, a.maskB) << a.s);
        if constexpr (E == EL_U64) {
            uint64_t acc = 0;
            for (uint64_t z = lane; z < K; z += 64) acc += ra[z] * rb[z];
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
            if (lane == 0) C[c] = acc;
        } else if constexpr (E == EL_I8) {
            int64_t acc = 0;
            if (K >= 1024) {
                // 16 bytes per lane and iteration (rows start 64-byte
                // aligned), four 4-way int8 dot products; a chunk's sum is at
                // most 16 127^2 < 2^18, widened once per chunk
                typedef int v4i_t __attribute__((ext_vector_type(4)));
                const v4i_t* va = reinterpret_cast<const v4i_t*>(ra);
                const v4i_t* vb = reinterpret_cast<const v4i_t*>(rb);
                for (uint64_t z = lane; z < K / 16; z += 64) {
                    const v4i_t x = va[z], y = vb[z];
                    int d = __builtin_amdgcn_sdot4(x[0], y[0], 0, false);
                    d = __builtin_amdgcn_sdot4(x[1], y[1], d, false);
                    d = __builtin_amdgcn_sdot4(x[2], y[2], d, false);
                    d = __builtin_amdgcn_sdot4(x[3], y[3], d, false);
                    acc += d;
                }
            } else {
                for (uint64_t z = lane; z < K; z += 64) acc += int32_t(ra[z]) * int32_t(rb[z]);
            }
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
            if (lane == 0) C[c] = T(ms.center64(acc));
        } else {
            uint64_t acc = 0;
            uint32_t n3 = 0;
            for (uint64_t z = lane; z < K; z += 64) {
                acc += uint64_t(ra[z]) * rb[z];
                if (++n3 == 3) {
                    acc = m.fold(acc);
                    n3 = 0;
                }
            }
            uint32_t r = m.finish(acc);
            for (int off = 32; off > 0; off >>= 1) {
                uint32_t o = __shfl_xor(r, off);
                uint32_t t = r + o;  // both < p < 2^31: no overflow
                r = t >= m.p ? t - m.p : t;
            }
            if (lane == 0) C[c] = r;
        }
    }
}

// Few outputs (2^rC <= 64), very wide K: the shared dimension is split over
// the grid. Block b sums its K slice for every output and writes one partial
// per output; a second kernel adds the partials of each output.

template <int E>
__global__ __launch_bounds__(256) void k_dot_partial(StepArgs a, uint64_t* scratch, int nblk) {
    using T = typename ElemT<E>::T;
    const void *pA, *pB;
    void* pC;
    load_planes<E>(a, pA, pB, pC);
    const T* A = static_cast<const T*>(pA);
    const T* B = static_cast<const T*>(pB);
    const ModP m{a.p[blockIdx.z], a.r2[blockIdx.z]};
    const ModSmall ms = mod_small(a);
    __shared__ uint64_t red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t K = uint64_t(1) << a.s;
    const uint64_t slice = K / uint64_t(nblk);
    const uint64_t z0 = slice * blockIdx.x;
    const uint64_t nOut = uint64_t(1) << a.rC;
    uint64_t* out = scratch + (uint64_t(blockIdx.z) * nblk + blockIdx.x) * 64;
    for (uint64_t c = 0; c < nOut; ++c) {
        const T* ra = A + (pext64(c, a.maskA) << a.s) + z0;
        const T* rb = B + (pext64(c, a.maskB) << a.s) + z0;
        uint64_t v;
        if constexpr (E == EL_U64) {
            uint64_t acc = 0;
            for (uint64_t z = threadIdx.x; z < slice; z += blockDim.x) acc += ra[z] * rb[z];
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
            v = acc;
        } else if constexpr (E == EL_I8) {
            int64_t acc = 0;
            for (uint64_t z = threadIdx.x; z < slice; z += blockDim.x) acc += int32_t(ra[z]) * int32_t(rb[z]);
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
            v = uint64_t(acc);
        } else {
            uint64_t acc = 0;
            uint32_t n3 = 0;
            for (uint64_t z = threadIdx.x; z < slice; z += blockDim.x) {
                acc += uint64_t(ra[z]) * rb[z];
                if (++n3 == 3) {
                    acc = m.fold(acc);
                    n3 = 0;
                }
            }
            uint32_t r = m.finish(acc);
            for (int o = 32; o > 0; o >>= 1) {
                const uint32_t t = r + __shfl_xor(r, o);
                r = t >= m.p ? t - m.p : t;
            }
            v = r;
        }
        if (lane == 0) red[wave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            if constexpr (E == EL_U64) {
                out[c] = red[0] + red[1] + red[2] + red[3];
            } else if constexpr (E == EL_I8) {
                // a centred residue, kept as a signed 64-bit value
                const int64_t t = int64_t(red[0]) + int64_t(red[1]) + int64_t(red[2]) + int64_t(red[3]);
                out[c] = uint64_t(int64_t(ms.center64(t)));
            } else {
                out[c] = (red[0] + red[1] + red[2] + red[3]) % m.p;
            }
        }
        __syncthreads();
    }
}

template <int E>
__global__ __launch_bounds__(64) void k_dot_final(StepArgs a, const uint64_t* scratch, int nblk) {
    using T = typename ElemT<E>::T;
    T* C = static_cast<T*>(a.C) + blockIdx.z * a.strideC;
    const uint32_t p = a.p[blockIdx.z];
    const ModSmall ms = mod_small(a);
    const uint64_t c = blockIdx.x;
    const uint64_t* part = scratch + uint64_t(blockIdx.z) * nblk * 64;
    uint64_t acc = 0;
    for (int b = threadIdx.x; b < nblk; b += 64) acc += part[uint64_t(b) * 64 + c];  // < 1024 * 2^31
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (threadIdx.x == 0) {
        if constexpr (E == EL_U64)
            C[c] = acc;
        else if constexpr (E == EL_I8)
            C[c] = T(ms.center64(int64_t(acc)));  // a sum of signed partials, in two's complement
        else
            C[c] = T(acc % p);
    }
}

// ----------------------------------------------------------------- launches

template <int E, int LOGK>
hipError_t launch_stream_nb(int nb, dim3 grid, hipStream_t st, const StepArgs& a) {
    switch (nb) {
        case 1: hipLaunchKernelGGL((k_stream<E, LOGK, 1>), grid, dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_stream<E, LOGK, 2>), grid, dim3(256), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_stream<E, LOGK, 4>), grid, dim3(256), 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_stream<E, LOGK, 8>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((k_stream<E, LOGK, 16>), grid, dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

template <int E>
hipError_t launch_stream(int logk, int nb, dim3 grid, hipStream_t st, const StepArgs& a) {
    switch (logk) {
        case 0: return launch_stream_nb<E, 0>(nb, grid, st, a);
        case 1: return launch_stream_nb<E, 1>(nb, grid, st, a);
        case 2: return launch_stream_nb<E, 2>(nb, grid, st, a);
        case 3: return launch_stream_nb<E, 3>(nb, grid, st, a);
        case 4: return launch_stream_nb<E, 4>(nb, grid, st, a);
        default: return launch_stream_nb<E, 5>(nb, grid, st, a);
    }
}

// launch of a kernel template instantiated per element kind
#define TN_LAUNCH_EL(el, kern, grid, block, stream, ...)                                     \
    do {                                                                                     \
        if ((el) == EL_U64)                                                                  \
            hipLaunchKernelGGL(kern<EL_U64>, grid, block, 0, stream, __VA_ARGS__);           \
        else if ((el) == EL_I8)                                                              \
            hipLaunchKernelGGL(kern<EL_I8>, grid, block, 0, stream, __VA_ARGS__);            \
        else                                                                                 \
            hipLaunchKernelGGL(kern<EL_U32>, grid, block, 0, stream, __VA_ARGS__);           \
    } while (0)

inline uint32_t cap32(uint64_t x, uint32_t hi) { return uint32_t(std::min<uint64_t>(std::max<uint64_t>(x, 1), hi)); }

// The streaming kernel with 2^nb B rows per thread (nb <= min(fB, 4)),
// without profiling (the autotuner's measurement launches).
hipError_t launch_stream_step(const StepArgs& a, int el, int G, int nb, hipStream_t st) {
    if (nb < 0 || nb > 4 || nb > a.fB || a.s > 5 || a.fA < 8) return hipErrorInvalidValue;
    const uint64_t n_iter = (uint64_t(1) << a.fA) >> 8;
    const uint64_t n_chunk = (uint64_t(1) << a.fB) >> nb;
    dim3 grid(cap32(n_iter, 1u << 20), cap32(n_chunk, 65535), uint32_t(G));
    return el == EL_U64  ? launch_stream<EL_U64>(a.s, 1 << nb, grid, st, a)
           : el == EL_I8 ? launch_stream<EL_I8>(a.s, 1 << nb, grid, st, a)
                         : launch_stream<EL_U32>(a.s, 1 << nb, grid, st, a);
}

KernelClass choose_class(const Step& st, int el, int flags) {
    StepArgs a{};
    a.s = st.s;
    a.rC = st.rC;
    a.fA = std::max(st.rA, st.rB) - st.s;  // the larger free side plays A
    a.fB = std::min(st.rA, st.rB) - st.s;
    if (flags & TN_FLAG_GENERIC_ONLY) return KC_GENERIC;
    if (a.rC <= 6 && a.s >= 10) return KC_DOT;
    if (el != EL_U64 && !st.initA && !st.initB && mfma_eligible(a, el) && !(flags & TN_FLAG_NO_MFMA)) return KC_MFMA;
    if (el == EL_I8 && narrow8_eligible(a) && !(flags & TN_FLAG_NO_MFMA)) return KC_NARROW;
    if (a.s <= 5 && a.fA >= 8) return KC_STREAM;
    if (a.s >= 6) return KC_ROWDOT;
    return KC_GENERIC;
}

std::vector<uint8_t> digit_plan(const Plan& plan, const std::vector<KernelClass>& cls, int el) {
    const size_t n = plan.steps.size();
    std::vector<uint8_t> out_dig(n, 0), dig(n, 0);
    if (el != EL_U32) return dig;  // int8 residues are the matrix-core operands as they are
    const size_t ids = size_t(plan.n_init) + n;
    std::vector<int32_t> prod(ids, -1), cons(ids, -1);
    for (size_t k = 0; k < n; ++k) {
        const Step& st = plan.steps[k];
        prod[size_t(st.out)] = int32_t(k);
        cons[size_t(st.a)] = int32_t(k);
        cons[size_t(st.b)] = int32_t(k);
    }
    for (size_t k = 0; k < n; ++k) {
        const int32_t c = cons[size_t(plan.steps[k].out)];
        out_dig[k] = cls[k] == KC_MFMA && c >= 0 && cls[size_t(c)] == KC_MFMA;
    }
    for (size_t k = 0; k < n; ++k) {
        const Step& st = plan.steps[k];
        const int32_t pa = prod[size_t(st.a)], pb = prod[size_t(st.b)];
        dig[k] = uint8_t((out_dig[k] ? 4 : 0) | (pa >= 0 && out_dig[size_t(pa)] ? 1 : 0) |
                         (pb >= 0 && out_dig[size_t(pb)] ? 2 : 0));
    }
    return dig;
}

int elem_size(int el) { return el == EL_U64 ? 8 : el == EL_I8 ? 1 : 4; }

void fill_moduli(StepArgs& a, const uint32_t* primes, int G) {
    for (int g = 0; g < G; ++g) {
        const uint32_t p = primes ? primes[g] : 0;
        a.p[g] = p;
        a.r2[g] = p ? uint32_t((uint64_t(1) << 32) % p) : 0;
        a.r16[g] = p ? uint32_t(65536u % p) : 0;
        a.pinv[g] = p ? 1.0f / float(p) : 0.0f;
    }
}

// Choose and launch the kernel of one step for a group of G residue planes.
hipError_t launch_step(const Step& st0, int el, int flags, const uint32_t* primes, int G, char* init_base,
                       char* arena_base, int64_t arena_elems, char* scratch, hipStream_t stream, KernelClass* kc,
                       int force, unsigned dig, int64_t init_stride) {
    const size_t es = size_t(elem_size(el));
    Profiler& prof = profiler();
    // algorithmic work of the step: entries read and written, multiply-adds
    const double step_bytes =
        double(es) * G * (std::ldexp(1.0, st0.rA) + std::ldexp(1.0, st0.rB) + std::ldexp(1.0, st0.rC));
    const double step_macs = double(G) * std::ldexp(1.0, st0.rA + st0.rB - st0.s);
    prof.cur_rA = st0.rA;
    prof.cur_rB = st0.rB;
    prof.cur_s = st0.s;
    prof.cur_rC = st0.rC;
    prof.cur_G = G;
    Step st = st0;
    StepArgs a{};
    a.B = st.initB ? init_base + st.offB * es : arena_base + st.offB * es;
    a.A = st.initA ? init_base + st.offA * es : arena_base + st.offA * es;
    a.C = arena_base + st.offC * es;
    a.strideA = st.initA ? init_stride : arena_elems;
    a.strideB = st.initB ? init_stride : arena_elems;
    a.strideC = arena_elems;
    const uint64_t cmask = st.rC >= 64 ? ~0ull : ((uint64_t(1) << st.rC) - 1);
    a.maskA = st.maskA;
    a.maskB = cmask & ~st.maskA;
    a.rC = st.rC;
    a.s = st.s;
    a.fA = st.rA - st.s;
    a.fB = st.rB - st.s;
    fill_moduli(a, primes, G);
    // the larger free side plays A
    if (a.fB > a.fA) {
        std::swap(a.A, a.B);
        std::swap(a.strideA, a.strideB);
        std::swap(a.maskA, a.maskB);
        std::swap(a.fA, a.fB);
        dig = (dig & 4u) | ((dig & 1u) << 1) | ((dig >> 1) & 1u);
    }
    const uint64_t total = uint64_t(1) << a.rC;
    const bool can_mfma = el != EL_U64 && !st.initA && !st.initB && mfma_eligible(a, el);
    const bool can_stream = a.s <= 5 && a.fA >= 8;
    if (force == KC_MFMA && !can_mfma) return hipErrorInvalidValue;
    if (force == KC_STREAM && !can_stream) return hipErrorInvalidValue;
    if (force == KC_ROWDOT && a.rC > 40) return hipErrorInvalidValue;
    const bool can_dot = a.rC <= 6 && a.s >= 10;
    if (force == KC_DOT && !can_dot) return hipErrorInvalidValue;
    if (force == KC_NARROW && !(el == EL_I8 && narrow8_eligible(a))) return hipErrorInvalidValue;
    // one decision rule for launches and for the digit-plane hand-over
    const int pick = force >= 0 ? force : int(choose_class(st0, el, flags));
    if (pick != KC_MFMA && (dig & 3u)) return hipErrorInvalidValue;  // operands must be plain residues
    if (pick == KC_DOT) {
        const int nblk = int(std::min<uint64_t>(kDotBlocks, (uint64_t(1) << a.s) >> 8));
        *kc = KC_DOT;
        dim3 g1(nblk, 1, G), g2(uint32_t(total), 1, G);
        uint64_t* scr = reinterpret_cast<uint64_t*>(scratch);
        prof.before(stream);
        TN_LAUNCH_EL(el, k_dot_partial, g1, dim3(256), stream, a, scr, nblk);
        prof.after_raw(stream, KC_DOT, step_bytes, step_macs);
        TN_LAUNCH_EL(el, k_dot_final, g2, dim3(64), stream, a, scr, nblk);
        return hipGetLastError();
    }
    if (pick == KC_NARROW) {
        *kc = KC_NARROW;
        return launch_narrow8(a, G, stream, &prof, step_bytes, step_macs, scratch, kScratchPerPrime);
    }
    if (pick == KC_MFMA) {
        *kc = KC_MFMA;
        if (el == EL_I8) return launch_mfma8(a, G, stream, &prof, step_bytes, step_macs, scratch, kScratchPerPrime);
        return launch_mfma(a, G, stream, &prof, step_bytes, step_macs, scratch, kScratchPerPrime, dig);
    }
    if (pick == KC_STREAM) {
        // B rows per thread: the autotuner's choice for the nearest tuned shape, else 2^min(fB, 4)
        const int tuned = tuned_choice(TK_STREAM, el, a.fA, a.fB, a.s);
        const int nb = tuned >= 0 ? std::min({tuned, a.fB, 4}) : std::min(a.fB, 4);
        const uint64_t n_iter = (uint64_t(1) << a.fA) >> 8;
        const uint64_t n_chunk = (uint64_t(1) << a.fB) >> nb;
        dim3 grid(cap32(n_iter, 1u << 20), cap32(n_chunk, 65535), G);
        *kc = KC_STREAM;
        prof.before(stream);
        hipError_t e = el == EL_U64  ? launch_stream<EL_U64>(a.s, 1 << nb, grid, stream, a)
                       : el == EL_I8 ? launch_stream<EL_I8>(a.s, 1 << nb, grid, stream, a)
                                     : launch_stream<EL_U32>(a.s, 1 << nb, grid, stream, a);
        prof.after_raw(stream, KC_STREAM, step_bytes, step_macs);
        return e;
    }
    if (pick == KC_ROWDOT) {
        dim3 grid(cap32((total + 3) / 4, 1u << 20), 1, G);
        *kc = KC_ROWDOT;
        prof.before(stream);
        TN_LAUNCH_EL(el, k_rowdot, grid, dim3(256), stream, a);
        prof.after_raw(stream, KC_ROWDOT, step_bytes, step_macs);
        return hipGetLastError();
    }
    dim3 grid(cap32((total + 255) / 256, 1u << 20), 1, G);
    *kc = KC_GENERIC;
    prof.before(stream);
    TN_LAUNCH_EL(el, k_generic, grid, dim3(256), stream, a);
    prof.after_raw(stream, KC_GENERIC, step_bytes, step_macs);
    return hipGetLastError();
}

// Value of one initial tensor entry x in the plan's bit order ``layout``
// (Eq. 3, Eq. 4, Eq. 6, parity; a negated index is reversed, Sec. 2.1; a
// table lists its entries by its own bond order).
uint64_t init_entry(const InitTensor& t, const std::vector<int32_t>& pos, uint64_t x) {
    const int r = int(t.bonds.size());
    if (t.kind == T_TABLE) {
        uint64_t own = 0;
        for (int k = 0; k < r; ++k) own |= ((x >> pos[k]) & 1) << k;
        return t.table[size_t(own)];
    }
    if (t.kind == T_COPY) {
        if (r == 0) return 2;  // a variable in no clause: both values count
        const uint64_t all = (r >= 64) ? ~0ull : ((uint64_t(1) << r) - 1);
        return (x == 0 || x == all) ? 1 : 0;
    }
    int ntrue = 0;
    for (int k = 0; k < r; ++k) {
        int bit = int((x >> pos[k]) & 1);
        ntrue += bit ^ int((t.neg >> k) & 1);
    }
    if (t.kind == T_OR) return ntrue >= 1 ? 1 : 0;
    if (t.kind == T_XOR) return uint64_t(ntrue & 1);
    return ntrue == 1 ? 1 : 0;
}

// Initial tensors in plan layout. Without moduli the raw entries are stored
// (entries of at most 127 are valid residues in every plane); with ``mod``
// (one modulus) each entry is reduced: centred for int8 planes.
void fill_init(const Network& net, const Plan& plan, int el, uint8_t* host, const uint32_t* mod) {
    for (int32_t i = 0; i < plan.n_init; ++i) {
        const InitTensor& t = net.t[i];
        const auto& L = plan.layout[i];
        std::vector<int32_t> pos(t.bonds.size());
        for (size_t k = 0; k < t.bonds.size(); ++k)
            pos[k] = int32_t(std::find(L.begin(), L.end(), t.bonds[k]) - L.begin());
        const uint64_t n = uint64_t(1) << t.bonds.size();
        for (uint64_t x = 0; x < n; ++x) {
            uint64_t v = init_entry(t, pos, x);
            if (el == EL_U64) {
                reinterpret_cast<uint64_t*>(host)[plan.init_off[i] + x] = v;
            } else if (el == EL_I8) {
                int32_t c = int32_t(v);
                if (mod) {
                    const int32_t m = int32_t(*mod), rr = int32_t(v % uint64_t(m));
                    c = rr > m / 2 ? rr - m : rr;
                }
                reinterpret_cast<int8_t*>(host)[plan.init_off[i] + x] = int8_t(c);
            } else {
                reinterpret_cast<uint32_t*>(host)[plan.init_off[i] + x] = uint32_t(mod ? v % *mod : v);
            }
        }
    }
}

// Whether the initial entries must be reduced per residue plane: an int8
// plane holds raw entries of at most 127 (any modulus), a u32 plane entries
// below its prime.
bool init_per_plane(const Plan& plan, const Resolved& R) {
    if (R.u64) return false;
    if (R.i8) return plan.max_entry > 127;
    return plan.max_entry >= *std::min_element(R.primes.begin(), R.primes.end());
}

tn_status resolve(const Plan& plan, const tn_contract_opts* o, Resolved& r) {
    int32_t arith = o ? o->arith : TN_ARITH_AUTO;
    if (arith == TN_ARITH_AUTO) arith = plan.count_bits <= 63 ? TN_ARITH_U64 : TN_ARITH_RNS;
    if (arith == TN_ARITH_U64) {
        if (plan.count_bits > 63) return TN_EINVAL;  // 64-bit wrapping is exact only below 2^64
        r.u64 = true;
        r.k = 1;
        return TN_OK;
    }
    if (arith != TN_ARITH_RNS) return TN_EINVAL;
    r.u64 = false;
    // small moduli (int8 residues) unless a prime count is given, 16-bit
    // primes are asked for, or the count needs more bits than they hold
    const int32_t ks = small_moduli_needed(plan.count_bits);
    if (!(o && o->n_primes > 0) && !(o && (o->flags & TN_FLAG_WIDE_RNS)) && ks > 0) {
        r.i8 = true;
        r.k = ks;
        const auto& M = small_moduli();
        r.primes.assign(M.begin(), M.begin() + ks);
        return TN_OK;
    }
    r.i8 = false;
    r.k = (o && o->n_primes > 0) ? o->n_primes : primes_needed(plan.count_bits);
    if (r.k > TN_MAX_PRIMES) return TN_EINVAL;
    const auto& P = prime_table(r.k);
    r.primes.assign(P.begin(), P.begin() + r.k);
    return TN_OK;
}

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// Runs the plan; fills residues (RNS) or *u64v (U64).
tn_status run_plan(const Network& net, const Plan& plan, const tn_contract_opts* o, const Resolved& R,
                   std::vector<uint32_t>& residues, uint64_t* u64v) {
    const int el = R.u64 ? EL_U64 : R.i8 ? EL_I8 : EL_U32;
    const size_t es = size_t(R.es());
    residues.assign(R.u64 ? 0 : R.k, 0);
    // networks that need no device work
    if (plan.n_init == 0) {
        if (R.u64) *u64v = 1;
        for (auto& x : residues) x = 1;
        return TN_OK;
    }
    if (plan.steps.empty()) {
        const InitTensor& t = net.t[plan.root];
        uint64_t v = init_entry(t, {}, 0);
        if (R.u64) *u64v = v;
        for (int i = 0; i < R.k && !R.u64; ++i) residues[i] = uint32_t(v % R.primes[i]);
        return TN_OK;
    }
    if (!o || !o->workspace) return TN_EINVAL;
    // initial tensors: one region for every plane, or one per plane of a
    // group when an entry needs reducing modulo each plane's modulus
    const bool pp = init_per_plane(plan, R);
    const int64_t init_bytes = align256(plan.init_elems * int64_t(es));
    const int64_t arena_bytes = align256(plan.arena_elems * int64_t(es));
    const int64_t arena_elems = arena_bytes / int64_t(es);
    const int64_t ws = int64_t(o->workspace_bytes);
    if (init_bytes + arena_bytes + kScratchPerPrime > ws) return TN_ETOOBIG;
    int G = pp ? int(ws / (init_bytes + arena_bytes + kScratchPerPrime))
               : int((ws - init_bytes) / (arena_bytes + kScratchPerPrime));
    G = std::min({G, R.k, kMaxGroup});
    if (o->prime_group > 0) G = std::min(G, int(o->prime_group));
    G = std::max(G, 1);
    hipStream_t stream = static_cast<hipStream_t>(o->stream);
    char* base = static_cast<char*>(o->workspace);
    char* init_base = base;
    char* arena_base = base + (pp ? int64_t(G) : 1) * init_bytes;
    char* scratch = arena_base + int64_t(G) * arena_bytes;
    const int64_t init_stride = pp ? init_bytes / int64_t(es) : 0;
    // host images: one region, or one per modulus (held until the end)
    const int n_img = pp ? R.k : 1;
    std::vector<uint8_t> host(size_t(init_bytes) * size_t(n_img), 0);
    for (int q = 0; q < n_img; ++q)
        fill_init(net, plan, el, host.data() + size_t(q) * size_t(init_bytes), pp ? &R.primes[size_t(q)] : nullptr);
    Profiler& prof = profiler();
    hipError_t err = pp ? hipSuccess : hipMemcpyAsync(init_base, host.data(), host.size(), hipMemcpyHostToDevice, stream);
    // on any failure, drain the stream before the host staging buffer goes away
    auto fail = [&]() {
        (void)hipStreamSynchronize(stream);
        prof.collect();
        return TN_EHIP;
    };
    if (err != hipSuccess) return fail();
    const Step& last = plan.steps.back();
    std::vector<KernelClass> cls(plan.steps.size());
    for (size_t k = 0; k < cls.size(); ++k) cls[k] = choose_class(plan.steps[k], el, o->flags);
    const std::vector<uint8_t> dig = digit_plan(plan, cls, el);
    std::vector<uint64_t> out(size_t(R.k), 0);
    for (int g0 = 0; g0 < R.k; g0 += G) {
        const int gn = std::min(G, R.k - g0);
        if (pp) {
            // this group's planes of the initial tensors
            err = hipMemcpyAsync(init_base, host.data() + size_t(g0) * size_t(init_bytes),
                                 size_t(gn) * size_t(init_bytes), hipMemcpyHostToDevice, stream);
            if (err != hipSuccess) return fail();
        }
        for (size_t k = 0; k < plan.steps.size(); ++k) {
            KernelClass kc = KC_GENERIC;
            err = launch_step(plan.steps[k], el, o->flags, R.u64 ? nullptr : R.primes.data() + g0, gn, init_base,
                              arena_base, arena_elems, scratch, stream, &kc, -1, dig[k], init_stride);
            if (err != hipSuccess) return fail();
        }
        for (int g = 0; g < gn; ++g) {
            err = hipMemcpyAsync(&out[g0 + g], arena_base + (g * arena_elems + last.offC) * int64_t(es), es,
                                 hipMemcpyDeviceToHost, stream);
            if (err != hipSuccess) return fail();
        }
    }
    err = hipStreamSynchronize(stream);
    if (err != hipSuccess) return TN_EHIP;
    prof.collect();
    if (R.u64) {
        *u64v = out[0];
    } else if (R.i8) {
        // a centred int8 residue in the low byte
        for (int i = 0; i < R.k; ++i) {
            const int32_t m = int32_t(R.primes[size_t(i)]), c = int32_t(int8_t(out[i] & 0xffu));
            residues[i] = uint32_t(c < 0 ? c + m : c);
        }
    } else {
        for (int i = 0; i < R.k; ++i) residues[i] = uint32_t(out[i] & 0xffffffffu);
    }
    return TN_OK;
}

}  // namespace tn

using namespace tn;

extern "C" {

tn_status tn_workspace_bytes(const tn_network* net, const tn_plan* plan, const tn_contract_opts* opts,
                             size_t* bytes) {
    if (!net || !plan || !bytes) return TN_EINVAL;
    Resolved R;
    tn_status st = resolve(plan->plan, opts, R);
    if (st != TN_OK) return st;
    const int64_t es = R.es();
    int G = (opts && opts->prime_group > 0) ? std::min<int>(opts->prime_group, std::min(R.k, kMaxGroup)) : 1;
    const int64_t init = align256(plan->plan.init_elems * es);
    *bytes = size_t((init_per_plane(plan->plan, R) ? int64_t(G) : 1) * init +
                    int64_t(G) * (align256(plan->plan.arena_elems * es) + kScratchPerPrime));
    return TN_OK;
}

tn_status tn_moduli(const tn_plan* plan, const tn_contract_opts* opts, uint32_t* out, int32_t cap, int32_t* k) {
    if (!plan || !k) return TN_EINVAL;
    Resolved R;
    tn_status st = resolve(plan->plan, opts, R);
    if (st != TN_OK) return st;
    *k = R.u64 ? 0 : R.k;
    if (R.u64) return TN_OK;
    if (!out || cap < R.k) return TN_EBUFSIZE;
    std::copy(R.primes.begin(), R.primes.end(), out);
    return TN_OK;
}

tn_status tn_contract(const tn_network* net, const tn_plan* plan, const tn_contract_opts* opts, uint32_t* residues,
                      int32_t residues_cap, uint64_t* u64) {
    if (!net || !plan) return TN_EINVAL;
    if (int32_t(net->net.t.size()) != plan->plan.n_init) return TN_EINVAL;
    Resolved R;
    tn_status st = resolve(plan->plan, opts, R);
    if (st != TN_OK) return st;
    if (!R.u64 && residues && residues_cap < R.k) return TN_EBUFSIZE;
    std::vector<uint32_t> res;
    uint64_t v = 0;
    profiler().start(opts && (opts->flags & TN_FLAG_TIMING));
    try {
        st = run_plan(net->net, plan->plan, opts, R, res, &v);
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    if (st != TN_OK) return st;
    if (R.u64) {
        if (u64) *u64 = v;
    } else if (residues) {
        std::copy(res.begin(), res.end(), residues);
    }
    return TN_OK;
}

tn_status tn_count(const tn_network* net, const tn_plan* plan, const tn_contract_opts* opts, uint32_t* limbs,
                   size_t cap, size_t* n_limbs) {
    if (!net || !plan || !n_limbs) return TN_EINVAL;
    if (int32_t(net->net.t.size()) != plan->plan.n_init) return TN_EINVAL;
    Resolved R;
    tn_status st = resolve(plan->plan, opts, R);
    if (st != TN_OK) return st;
    std::vector<uint32_t> res, L;
    uint64_t v = 0;
    profiler().start(opts && (opts->flags & TN_FLAG_TIMING));
    try {
        st = run_plan(net->net, plan->plan, opts, R, res, &v);
        if (st != TN_OK) return st;
        if (R.u64) {
            L = {uint32_t(v), uint32_t(v >> 32)};
            while (L.size() > 1 && L.back() == 0) L.pop_back();
        } else {
            crt_limbs(res.data(), R.primes.data(), R.k, L);
        }
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    *n_limbs = L.size();
    if (!limbs || cap < L.size()) return TN_EBUFSIZE;
    std::copy(L.begin(), L.end(), limbs);
    return TN_OK;
}

}  // extern "C"

// ------------------------------------------------- allocation-free variant
// Device memory for tn_contract_noalloc: one file-scope array per GPU (each
// device that loads the library holds its own copy until the process ends).
// Host code never passes the array's name to a kernel or a copy: it looks up
// the array's device address once per device (hipGetSymbolAddress, with that
// device current) and uses that address as the workspace.
static constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

tn_status noalloc_workspace(void** ptr) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TN_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TN_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return TN_OK;
}
}  // namespace

extern "C" tn_status tn_contract_noalloc(const tn_network* net, const tn_plan* plan, const tn_contract_opts* opts,
                                         uint32_t* residues, int32_t residues_cap, uint64_t* u64) {
    if (!net || !plan || !opts) return TN_EINVAL;
    // per-launch timing creates events: not available without allocation
    if (opts->flags & TN_FLAG_TIMING) return TN_EUNSUPPORTED;
    tn_contract_opts o = *opts;
    void* ws = nullptr;
    const tn_status st = noalloc_workspace(&ws);
    if (st != TN_OK) return st;
    o.workspace = ws;
    o.workspace_bytes = kNoAllocBytes;
    // the plan's init region, arena and scratch must fit the array; run_plan
    // returns TN_ETOOBIG before any device work otherwise
    return tn_contract(net, plan, &o, residues, residues_cap, u64);
}

extern "C" size_t tn_noalloc_max_bytes(void) { return kNoAllocBytes; }

extern "C" tn_status tn_step(const void* A, int32_t rA, const void* B, int32_t rB, int32_t s, uint64_t maskA,
                             int32_t arith, uint32_t prime, int32_t kernel, void* C, void* workspace,
                             size_t workspace_bytes, void* stream_) {
    if (!A || !B || !C || !workspace) return TN_EINVAL;
    if (rA < 0 || rB < 0 || s < 0 || s > rA || s > rB) return TN_EINVAL;
    const int32_t rC = rA + rB - 2 * s;
    if (rA > TN_MAX_RANK || rB > TN_MAX_RANK || rC > TN_MAX_RANK) return TN_ERANK;
    const uint64_t cmask = (uint64_t(1) << rC) - 1;
    if ((maskA & ~cmask) || __builtin_popcountll(maskA) != rA - s) return TN_EINVAL;
    const bool u64 = arith == TN_ARITH_U64;
    // residues: modulo an odd prime in (2^16 - 2^11, 65280), or modulo a
    // small modulus 2 <= m <= 255 (held as centred int8 on the device)
    const bool small = !u64 && prime >= 2 && prime <= kSmallModulusMax;
    if (!u64 && !small &&
        (arith != TN_ARITH_RNS || prime <= 65536u - 2048u || prime >= kPrimeBound || prime % 2 == 0))
        return TN_EINVAL;
    if (small && arith != TN_ARITH_RNS) return TN_EINVAL;
    if (kernel < -1 || kernel > KC_NARROW || kernel == KC_BATCH || kernel == KC_DIGITS) return TN_EINVAL;
    const int el = u64 ? EL_U64 : small ? EL_I8 : EL_U32;
    const int64_t es = elem_size(el);
    const int64_t nA = align256((int64_t(1) << rA) * es), nB = align256((int64_t(1) << rB) * es),
                  nC = align256((int64_t(1) << rC) * es);
    if (nA + nB + nC + kScratchPerPrime > int64_t(workspace_bytes)) return TN_ETOOBIG;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    char* base = static_cast<char*>(workspace);
    Step st;
    st.rA = rA;
    st.rB = rB;
    st.s = s;
    st.rC = rC;
    st.maskA = maskA;
    st.initA = st.initB = false;
    st.offA = 0;
    st.offB = nA / es;
    st.offC = (nA + nB) / es;
    // small moduli: host residues in [0, m) as u32 <-> centred int8
    std::vector<int8_t> a8, b8, c8;
    const void* srcA = A;
    const void* srcB = B;
    if (small) {
        const int32_t m = int32_t(prime);
        auto centre = [m](const uint32_t* x, int64_t n, std::vector<int8_t>& out) {
            out.resize(size_t(n));
            for (int64_t i = 0; i < n; ++i) {
                const int32_t r = int32_t(x[i] % uint32_t(m));
                out[size_t(i)] = int8_t(r > m / 2 ? r - m : r);
            }
        };
        centre(static_cast<const uint32_t*>(A), int64_t(1) << rA, a8);
        centre(static_cast<const uint32_t*>(B), int64_t(1) << rB, b8);
        c8.resize(size_t(int64_t(1) << rC));
        srcA = a8.data();
        srcB = b8.data();
    }
    if (hipMemcpyAsync(base, srcA, size_t((int64_t(1) << rA) * es), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(base + nA, srcB, size_t((int64_t(1) << rB) * es), hipMemcpyHostToDevice, stream) !=
            hipSuccess) {
        (void)hipStreamSynchronize(stream);
        return TN_EHIP;
    }
    KernelClass kc = KC_GENERIC;
    hipError_t e = launch_step(st, el, 0, u64 ? nullptr : &prime, 1, base, base, 0, base + nA + nB + nC, stream, &kc,
                               kernel);
    if (e == hipErrorInvalidValue) {
        (void)hipStreamSynchronize(stream);
        return TN_EUNSUPPORTED;
    }
    void* dstC = small ? static_cast<void*>(c8.data()) : C;
    if (e != hipSuccess ||
        hipMemcpyAsync(dstC, base + nA + nB, size_t((int64_t(1) << rC) * es), hipMemcpyDeviceToHost, stream) !=
            hipSuccess) {
        (void)hipStreamSynchronize(stream);
        return TN_EHIP;
    }
    if (hipStreamSynchronize(stream) != hipSuccess) return TN_EHIP;
    if (small) {
        const int32_t m = int32_t(prime);
        uint32_t* out = static_cast<uint32_t*>(C);
        for (int64_t i = 0; i < (int64_t(1) << rC); ++i) {
            const int32_t c = c8[size_t(i)];
            out[i] = uint32_t(c < 0 ? c + m : c);
        }
    }
    return TN_OK;
}

namespace tn {
Profiler& profiler() {
    static thread_local Profiler p;
    return p;
}
}  // namespace tn

extern "C" tn_status tn_profile_launches(tn_launch_record* out, int64_t cap, int64_t* n) {
    if (!n) return TN_EINVAL;
    const auto& r = tn::profiler().recs;
    *n = int64_t(r.size());
    if (!out) return TN_OK;
    if (cap < int64_t(r.size())) return TN_EBUFSIZE;
    std::copy(r.begin(), r.end(), out);
    return TN_OK;
}

extern "C" tn_status tn_profile_get(tn_kernel_profile* out) {
    if (!out) return TN_EINVAL;
    for (int i = 0; i < TN_KERNEL_CLASSES; ++i) out[i] = tn::profiler().acc[i];
    return TN_OK;
}
