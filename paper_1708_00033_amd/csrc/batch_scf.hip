// Batched SCF steps on padded per-molecule slots.
//
// A batch's molecules have different basis sizes n_m <= NP.  For the SCF
// steps around the Fock build (energy, DIIS error and extrapolation,
// projection, eigensolve, density) every molecule owns one NP x NP slot
// (column-major, zero outside its n_m x n_m or n_m x k_m block), so that each
// step is one launch for the whole batch: uniform strided-batched GEMMs and
// the kernels below.  The zero padding leaves every product's physical block
// unchanged.  All launches take device-resident parameters (ring slots,
// DIIS coefficients, active flags), so a captured sequence stays valid from
// one SCF iteration to the next.
#include <hip/hip_runtime.h>

#define BS_WG 256

namespace {

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[BS_WG / 64];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BS_WG / 64; ++w) s += red[w];
    return s;   // valid on thread 0
}

// slot[m] (NP x NP, column-major) <- ragged row-major block of molecule m
// (symmetric matrices: the two layouts coincide on the block)
__global__ void k_pack(const double* __restrict__ rag, const long long* __restrict__ moff,
                       const int* __restrict__ dim, int NP, double* __restrict__ pad) {
    const int m = blockIdx.y, n = dim[m];
    const size_t tot = (size_t)NP * NP;
    double* __restrict__ d = pad + (size_t)m * tot;
    for (size_t x = (size_t)blockIdx.x * BS_WG + threadIdx.x; x < tot; x += (size_t)gridDim.x * BS_WG) {
        const int col = (int)(x / NP), row = (int)(x % NP);
        d[x] = (row < n && col < n) ? rag[moff[m] + (size_t)row * n + col] : 0.0;
    }
}

// E_m = sum over molecule m's block of D (H + F)
__global__ void k_energy_m(const double* __restrict__ D, const double* __restrict__ H, const double* __restrict__ F,
                           const long long* __restrict__ moff, const int* __restrict__ dim, double* __restrict__ E) {
    const int m = blockIdx.x;
    const size_t nn = (size_t)dim[m] * dim[m], o = (size_t)moff[m];
    double acc = 0.0;
    for (size_t x = threadIdx.x; x < nn; x += BS_WG) acc += D[o + x] * (H[o + x] + F[o + x]);
    acc = block_sum(acc);
    if (threadIdx.x == 0) E[m] = acc;
}

// out = A - A^T per slot
__global__ void k_antisym_pad(const double* __restrict__ A, int NP, double* __restrict__ out) {
    const int m = blockIdx.y;
    const size_t tot = (size_t)NP * NP;
    const double* __restrict__ a = A + (size_t)m * tot;
    double* __restrict__ o = out + (size_t)m * tot;
    for (size_t x = (size_t)blockIdx.x * BS_WG + threadIdx.x; x < tot; x += (size_t)gridDim.x * BS_WG) {
        const size_t col = x / NP, row = x % NP;
        o[x] = a[x] - a[row * NP + col];
    }
}

// ring[m][slot[m]] <- src[m] for the molecules with slot[m] >= 0
__global__ void k_ring_store(const double* __restrict__ src, int NP, const int* __restrict__ slot, int dmax,
                             double* __restrict__ ring) {
    const int m = blockIdx.y, sl = slot[m];
    if (sl < 0) return;
    const size_t tot = (size_t)NP * NP;
    const double* __restrict__ s = src + (size_t)m * tot;
    double* __restrict__ d = ring + ((size_t)m * dmax + sl) * tot;
    for (size_t x = (size_t)blockIdx.x * BS_WG + threadIdx.x; x < tot; x += (size_t)gridDim.x * BS_WG) d[x] = s[x];
}

// dots[m * dmax + i] = <e[m], ring[m][i]> for every ring slot i
__global__ void k_ring_dots(const double* __restrict__ e, const double* __restrict__ ring, int NP, int dmax,
                            double* __restrict__ dots) {
    const int m = blockIdx.y, i = blockIdx.x;
    const size_t tot = (size_t)NP * NP;
    const double* __restrict__ a = e + (size_t)m * tot;
    const double* __restrict__ b = ring + ((size_t)m * dmax + i) * tot;
    double acc = 0.0;
    for (size_t x = threadIdx.x; x < tot; x += BS_WG) acc += a[x] * b[x];
    acc = block_sum(acc);
    if (threadIdx.x == 0) dots[(size_t)m * dmax + i] = acc;
}

// out[m] = sum_i coef[m * dmax + i] ring[m][i]
__global__ void k_ring_lincomb(const double* __restrict__ ring, const double* __restrict__ coef, int NP, int dmax,
                               double* __restrict__ out) {
    const int m = blockIdx.y;
    const size_t tot = (size_t)NP * NP;
    const double* __restrict__ c = coef + (size_t)m * dmax;
    double* __restrict__ o = out + (size_t)m * tot;
    for (size_t x = (size_t)blockIdx.x * BS_WG + threadIdx.x; x < tot; x += (size_t)gridDim.x * BS_WG) {
        double v = 0.0;
        for (int i = 0; i < dmax; ++i) {
            const double ci = c[i];
            if (ci != 0.0) v += ci * ring[((size_t)m * dmax + i) * tot + x];
        }
        o[x] = v;
    }
}

// Keep the first nocc[m] columns of slot m (the occupied orbitals), zero the rest.
__global__ void k_occ_cols(const double* __restrict__ C, const int* __restrict__ nocc, int NP,
                           double* __restrict__ out) {
    const int m = blockIdx.y, no = nocc[m];
    const size_t tot = (size_t)NP * NP;
    for (size_t x = (size_t)blockIdx.x * BS_WG + threadIdx.x; x < tot; x += (size_t)gridDim.x * BS_WG) {
        const int col = (int)(x / NP);
        out[(size_t)m * tot + x] = col < no ? C[(size_t)m * tot + x] : 0.0;
    }
}

// sq[m] = sum over the n_m x n_m block of (Dn - D)^2
__global__ void k_dsq(const double* __restrict__ Dn, const double* __restrict__ D, const int* __restrict__ dim, int NP,
                      double* __restrict__ sq) {
    const int m = blockIdx.x, n = dim[m];
    const size_t tot = (size_t)NP * NP;
    double acc = 0.0;
    for (size_t x = threadIdx.x; x < (size_t)n * n; x += BS_WG) {
        const size_t col = x / n, row = x % n, k = (size_t)m * tot + col * NP + row;
        const double d = Dn[k] - D[k];
        acc += d * d;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) sq[m] = acc;
}

// For active molecules: D_pad <- Dn_pad and the ragged density <- its block.
__global__ void k_take_density(const double* __restrict__ Dn, const int* __restrict__ active,
                               const long long* __restrict__ moff, const int* __restrict__ dim, int NP,
                               double* __restrict__ Dpad, double* __restrict__ rag) {
    const int m = blockIdx.y;
    if (!active[m]) return;
    const int n = dim[m];
    const size_t tot = (size_t)NP * NP;
    for (size_t x = (size_t)blockIdx.x * BS_WG + threadIdx.x; x < tot; x += (size_t)gridDim.x * BS_WG) {
        const double v = Dn[(size_t)m * tot + x];
        Dpad[(size_t)m * tot + x] = v;
        const int col = (int)(x / NP), row = (int)(x % NP);
        if (row < n && col < n) rag[moff[m] + (size_t)row * n + col] = v;
    }
}

dim3 slot_grid(int NP, int nmol) {
    size_t g = ((size_t)NP * NP + BS_WG - 1) / BS_WG;
    if (g > 1024) g = 1024;
    return dim3((unsigned)(g ? g : 1), (unsigned)nmol);
}

}  // namespace

extern "C" {
hipError_t hfx_bscf_pack(const double* rag, const long long* moff, const int* dim, int nmol, int NP, double* pad,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_pack, slot_grid(NP, nmol), dim3(BS_WG), 0, st, rag, moff, dim, NP, pad);
    return hipGetLastError();
}
hipError_t hfx_bscf_energy(const double* D, const double* H, const double* F, const long long* moff, const int* dim,
                           int nmol, double* E, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_m, dim3(nmol), dim3(BS_WG), 0, st, D, H, F, moff, dim, E);
    return hipGetLastError();
}
hipError_t hfx_bscf_antisym(const double* A, int nmol, int NP, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_antisym_pad, slot_grid(NP, nmol), dim3(BS_WG), 0, st, A, NP, out);
    return hipGetLastError();
}
hipError_t hfx_bscf_ring_store(const double* src, int nmol, int NP, const int* slot, int dmax, double* ring,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_ring_store, slot_grid(NP, nmol), dim3(BS_WG), 0, st, src, NP, slot, dmax, ring);
    return hipGetLastError();
}
hipError_t hfx_bscf_ring_dots(const double* e, const double* ring, int nmol, int NP, int dmax, double* dots,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_ring_dots, dim3(dmax, nmol), dim3(BS_WG), 0, st, e, ring, NP, dmax, dots);
    return hipGetLastError();
}
hipError_t hfx_bscf_ring_lincomb(const double* ring, const double* coef, int nmol, int NP, int dmax, double* out,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_ring_lincomb, slot_grid(NP, nmol), dim3(BS_WG), 0, st, ring, coef, NP, dmax, out);
    return hipGetLastError();
}
hipError_t hfx_bscf_occ_cols(const double* C, const int* nocc, int nmol, int NP, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_occ_cols, slot_grid(NP, nmol), dim3(BS_WG), 0, st, C, nocc, NP, out);
    return hipGetLastError();
}
hipError_t hfx_bscf_dsq(const double* Dn, const double* D, const int* dim, int nmol, int NP, double* sq,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_dsq, dim3(nmol), dim3(BS_WG), 0, st, Dn, D, dim, NP, sq);
    return hipGetLastError();
}
hipError_t hfx_bscf_take_density(const double* Dn, const int* active, const long long* moff, const int* dim, int nmol,
                                 int NP, double* Dpad, double* rag, hipStream_t st) {
    hipLaunchKernelGGL(k_take_density, slot_grid(NP, nmol), dim3(BS_WG), 0, st, Dn, active, moff, dim, NP, Dpad,
                       rag);
    return hipGetLastError();
}
}
