// cns_spectrum.hip -- kinetic-energy spectrum E(k) of a state on the GPU.
//
// The paper characterises its decaying-turbulence runs by the energy spectrum (Sec. 2.3:
// the model initial spectrum and the spectrum at t/tau = 3; Sec. 5: spectra per grid
// size) and by the Taylor microscale lambda behind Re_lambda and tau = lambda/u0.  Here
//   v_hat(k) = (1/N) sum_x v(x) exp(-i k.x),  N = nx ny nz,  v = m/rho,
//   E(k_s)   = sum over modes with round(|k|) = k_s of |v_hat|^2 / 2  (unit-width shells),
//   M2       = sum over all modes of |k|^2 |v_hat|^2 / 2,
// with the physical wavenumber k_d = 2 pi n_d / L_d.
//
// Steps (all on the plan's stream, FP64 whatever the plan's precision):
//   1. pack: X1 = v_x + i v_y, X2 = v_z.  Two real fields share one complex transform;
//      the shells are symmetric under k -> -k, so sum_shell |X|^2 equals the sum of the
//      two real fields' |v_hat|^2 without separating them.
//   2. three passes of batched 1-D FFTs (x, then y, then z), each line staged in LDS and
//      transformed by a mixed-radix Stockham autosort FFT (radix 4, 2 and 3, 5, ... as
//      generic small-prime butterflies), lines of the y and z passes batched along x so
//      loads and stores stay coalesced.
//   3. binning: per-block shell histograms in LDS, then a fixed-order sum over blocks
//      (one block per shell) and over shells.
//      (LDS double atomics: the last bits of a shell sum may vary between runs.)
// Scratch: the plan's stage buffers A (X1), B (X2) and rhs (block partials).
#include <cmath>
#include <vector>

#include "cns_internal.h"

namespace cns {

constexpr int kFftThreads = 256;
constexpr int kFftMaxRadix = 32;
constexpr size_t kFftLdsMax = 64 * 1024;

struct FftPlan {
    int N;            // line length
    int nr;           // number of radix stages
    int radix[kFftMaxRadix];
    long long nlines;
    int nl;           // lines per block
    int ld;           // LDS stride between lines (N + 1: consecutive lines fall in different banks)
    long long na;     // line index L -> (L % na) * sa + (L / na) * sb
    size_t sa, sb, es;
    int contig;       // 1: elements of a line are contiguous (x pass)
};

template <typename T>
__global__ void k_spec_pack(const T *u, size_t n3, double2 *X1, double2 *X2) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n3; i += (size_t)gridDim.x * blockDim.x) {
        const double r = double(u[i]);
        const double vx = double(u[n3 + i]) / r, vy = double(u[2 * n3 + i]) / r, vz = double(u[3 * n3 + i]) / r;
        X1[i] = make_double2(vx, vy);
        X2[i] = make_double2(vz, 0.0);
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// exp(-2 pi i num / den) (forward transform)
__device__ __forceinline__ double2 twiddle(long long num, long long den) {
    double s, c;
    sincospi(-2.0 * (double)num / (double)den, &s, &c);
    return make_double2(c, s);
}

// One Stockham stage of radix R on nl lines of length N: src -> dst (LDS), Ns = product of
// the radices of the earlier stages.  Butterfly j (0 <= j < N/R) reads src[j + r N/R],
// r = 0..R-1, applies the twiddles exp(-2 pi i r k/(Ns R)) with k = j mod Ns, takes a
// length-R DFT and writes output s to dst[(j/Ns) Ns R + k + s Ns].
template <int R>
__device__ __forceinline__ void fft_stage_small(const double2 *src, double2 *dst, int N, int ld, int nl, int Ns) {
    const int m = N / R;
    for (int t = threadIdx.x; t < nl * m; t += blockDim.x) {
        const int l = t / m, j = t % m;
        const double2 *a = src + (size_t)l * ld;
        double2 *b = dst + (size_t)l * ld;
        const int k = j % Ns;
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            v[r] = a[j + r * m];
            if (r) v[r] = cmul(v[r], twiddle((long long)r * k, (long long)Ns * R));
        }
        const int o = (j / Ns) * Ns * R + k;
        if constexpr (R == 2) {
            b[o] = cadd(v[0], v[1]);
            b[o + Ns] = csub(v[0], v[1]);
        } else if constexpr (R == 4) {
            const double2 s0 = cadd(v[0], v[2]), d0 = csub(v[0], v[2]);
            const double2 s1 = cadd(v[1], v[3]), d1 = csub(v[1], v[3]);
            const double2 md1 = make_double2(d1.y, -d1.x);  // -i * d1
            b[o] = cadd(s0, s1);
            b[o + Ns] = cadd(d0, md1);
            b[o + 2 * Ns] = csub(s0, s1);
            b[o + 3 * Ns] = csub(d0, md1);
        } else {
#pragma unroll
            for (int s = 0; s < R; ++s) {
                double2 acc = v[0];
#pragma unroll
                for (int r = 1; r < R; ++r) acc = cadd(acc, cmul(v[r], twiddle((long long)((r * s) % R), R)));
                b[o + s * Ns] = acc;
            }
        }
    }
}

// generic radix R (any prime): one work item per output
__device__ __forceinline__ void fft_stage_generic(const double2 *src, double2 *dst, int N, int ld, int nl, int Ns,
                                                  int R) {
    const int m = N / R;
    for (int t = threadIdx.x; t < nl * N; t += blockDim.x) {
        const int l = t / N, q = t % N;
        const int j = q % m, s = q / m;
        const double2 *a = src + (size_t)l * ld;
        const int k = j % Ns;
        double2 acc = a[j];
        for (int r = 1; r < R; ++r) {
            const double2 v = cmul(a[j + r * m], twiddle((long long)r * k, (long long)Ns * R));
            acc = cadd(acc, cmul(v, twiddle((long long)((r * s) % R), R)));
        }
        dst[(size_t)l * ld + (j / Ns) * Ns * R + k + s * Ns] = acc;
    }
}

__global__ __launch_bounds__(kFftThreads) void k_fft_lines(double2 *data, FftPlan P) {
    extern __shared__ double2 lds_c[];
    const int N = P.N, nl = P.nl, ld = P.ld;
    for (long long g = blockIdx.x; g * nl < P.nlines; g += gridDim.x) {
        const long long L0 = g * nl;
        const int nact = (int)min((long long)nl, P.nlines - L0);
        double2 *src = lds_c, *dst = lds_c + (size_t)nl * ld;
        for (int t = threadIdx.x; t < nl * N; t += blockDim.x) {
            const int l = P.contig ? t / N : t % nl;
            const int j = P.contig ? t % N : t / nl;
            if (l < nact) {
                const long long L = L0 + l;
                const size_t base = (size_t)(L % P.na) * P.sa + (size_t)(L / P.na) * P.sb;
                src[(size_t)l * ld + j] = data[base + (size_t)j * P.es];
            } else {
                src[(size_t)l * ld + j] = make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
        int Ns = 1;
        for (int st = 0; st < P.nr; ++st) {
            const int R = P.radix[st];
            if (R == 4) fft_stage_small<4>(src, dst, N, ld, nl, Ns);
            else if (R == 2) fft_stage_small<2>(src, dst, N, ld, nl, Ns);
            else if (R == 3) fft_stage_small<3>(src, dst, N, ld, nl, Ns);
            else if (R == 5) fft_stage_small<5>(src, dst, N, ld, nl, Ns);
            else fft_stage_generic(src, dst, N, ld, nl, Ns, R);
            __syncthreads();
            double2 *tmp = src;
            src = dst;
            dst = tmp;
            Ns *= R;
        }
        for (int t = threadIdx.x; t < nl * N; t += blockDim.x) {
            const int l = P.contig ? t / N : t % nl;
            const int j = P.contig ? t % N : t / nl;
            if (l < nact) {
                const long long L = L0 + l;
                const size_t base = (size_t)(L % P.na) * P.sa + (size_t)(L / P.na) * P.sb;
                data[base + (size_t)j * P.es] = src[(size_t)l * ld + j];
            }
        }
        __syncthreads();  // the next group reuses the LDS
    }
}

struct SpecGeom {
    int nx, ny, nz, nshell;
    size_t n3;
    double kux, kuy, kuz;  // 2 pi / L_d
    double norm;           // 1 / n3^2
};

__device__ __forceinline__ int signed_freq(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

__global__ __launch_bounds__(kPointThreads) void k_spec_bin(const double2 *X1, const double2 *X2, SpecGeom G,
                                                            double *part) {
    extern __shared__ double hist[];  // [2][nshell]: E, |k|^2 E
    for (int s = threadIdx.x; s < 2 * G.nshell; s += blockDim.x) hist[s] = 0.0;
    __syncthreads();
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < G.n3; i += (size_t)gridDim.x * blockDim.x) {
        const int ix = (int)(i % G.nx);
        const int iy = (int)((i / G.nx) % G.ny);
        const int iz = (int)(i / ((size_t)G.nx * G.ny));
        const double kx = signed_freq(ix, G.nx) * G.kux, ky = signed_freq(iy, G.ny) * G.kuy,
                     kz = signed_freq(iz, G.nz) * G.kuz;
        const double k2 = kx * kx + ky * ky + kz * kz;
        const int s = min((int)floor(sqrt(k2) + 0.5), G.nshell - 1);
        const double2 a = X1[i], b = X2[i];
        const double p = 0.5 * (a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y) * G.norm;
        atomicAdd(&hist[s], p);
        atomicAdd(&hist[G.nshell + s], k2 * p);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < 2 * G.nshell; s += blockDim.x) part[(size_t)blockIdx.x * 2 * G.nshell + s] = hist[s];
}

// E[s], M2[s] = sum over the block partials in a fixed order: one block per shell, its
// threads striding over the partials, then a fixed-shape tree in LDS
__global__ __launch_bounds__(kPointThreads) void k_spec_final(const double *part, int nblocks, int nshell, double *E,
                                                              double *M2) {
    __shared__ double re[kPointThreads], rm[kPointThreads];
    const int s = blockIdx.x;
    double e = 0.0, m = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        e += part[(size_t)b * 2 * nshell + s];
        m += part[(size_t)b * 2 * nshell + nshell + s];
    }
    re[threadIdx.x] = e;
    rm[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            re[threadIdx.x] += re[threadIdx.x + w];
            rm[threadIdx.x] += rm[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        E[s] = re[0];
        M2[s] = rm[0];
    }
}

// mom = {sum_s E[s], sum_s M2[s]} in shell order
__global__ void k_spec_mom(const double *E, const double *M2, int nshell, double *mom) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double e = 0.0, m = 0.0;
    for (int s = 0; s < nshell; ++s) {
        e += E[s];
        m += M2[s];
    }
    mom[0] = e;
    mom[1] = m;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int fft_factor(int n, int *radix) {
    int nr = 0;
    while (n % 4 == 0) radix[nr++] = 4, n /= 4;
    while (n % 2 == 0) radix[nr++] = 2, n /= 2;
    for (int p = 3; n > 1; p += 2)
        while (n % p == 0) radix[nr++] = p, n /= p;
    return nr;
}

int spectrum_shells(const BoxDesc &b) {
    const double kx = (b.nx / 2) * (2.0 * M_PI * b.inv_h[0] / b.nx);
    const double ky = (b.ny / 2) * (2.0 * M_PI * b.inv_h[1] / b.ny);
    const double kz = (b.nz / 2) * (2.0 * M_PI * b.inv_h[2] / b.nz);
    return (int)std::floor(std::sqrt(kx * kx + ky * ky + kz * kz) + 0.5) + 1;
}

bool spectrum_supported(const BoxDesc &b) {
    const int n[3] = {b.nx, b.ny, b.nz};
    for (int d = 0; d < 3; ++d)
        if ((size_t)2 * (n[d] + 1) * sizeof(double2) > kFftLdsMax) return false;
    // the shell histogram must fit in LDS, one block's partials and the per-shell second
    // moments in the rhs buffer (at least 20 bytes per point)
    const size_t hist = 2 * sizeof(double) * (size_t)spectrum_shells(b);
    return hist <= kFftLdsMax && hist + sizeof(double) * (size_t)spectrum_shells(b) <= 20 * b.n3;
}

static void fft_pass(double2 *X, const BoxDesc &b, int dir, hipStream_t s) {
    FftPlan P{};
    const size_t nx = b.nx, ny = b.ny, nz = b.nz;
    P.N = dir == 0 ? b.nx : (dir == 1 ? b.ny : b.nz);
    P.nr = fft_factor(P.N, P.radix);
    P.nlines = (long long)(b.n3 / P.N);
    if (dir == 0) {
        P.na = P.nlines, P.sa = nx, P.sb = 0, P.es = 1, P.contig = 1;
    } else if (dir == 1) {
        P.na = nx, P.sa = 1, P.sb = nx * ny, P.es = nx, P.contig = 0;
    } else {
        P.na = P.nlines, P.sa = 1, P.sb = 0, P.es = nx * ny, P.contig = 0;
    }
    // lines per block: fill the LDS budget (two buffers), at most 64 lines
    P.ld = P.N + 1;
    const int nl = (int)std::max<size_t>(1, std::min<size_t>(64, kFftLdsMax / (2 * sizeof(double2) * P.ld)));
    P.nl = nl;
    const size_t lds = 2 * sizeof(double2) * (size_t)nl * P.ld;
    const long long groups = (P.nlines + nl - 1) / nl;
    const unsigned grid = (unsigned)std::min<long long>(groups, 1 << 20);
    (void)nz;
    hipLaunchKernelGGL(k_fft_lines, dim3(grid), dim3(kFftThreads), lds, s, X, P);
}

void launch_spectrum(const BoxDesc &b, int prec, hipStream_t s, const void *u, double *E, int nshell, double *mom) {
    double2 *X1 = (double2 *)b.A, *X2 = (double2 *)b.B;
    const unsigned pg = (unsigned)std::min<size_t>((b.n3 + kPointThreads - 1) / kPointThreads, 65536);
    if (prec == CNS_FP64)
        hipLaunchKernelGGL(k_spec_pack<double>, dim3(pg), dim3(kPointThreads), 0, s, (const double *)u, b.n3, X1, X2);
    else
        hipLaunchKernelGGL(k_spec_pack<float>, dim3(pg), dim3(kPointThreads), 0, s, (const float *)u, b.n3, X1, X2);
    for (int d = 0; d < 3; ++d) {
        fft_pass(X1, b, d, s);
        fft_pass(X2, b, d, s);
    }
    SpecGeom G;
    G.nx = b.nx, G.ny = b.ny, G.nz = b.nz, G.nshell = nshell, G.n3 = b.n3;
    G.kux = 2.0 * M_PI * b.inv_h[0] / b.nx;
    G.kuy = 2.0 * M_PI * b.inv_h[1] / b.ny;
    G.kuz = 2.0 * M_PI * b.inv_h[2] / b.nz;
    G.norm = 1.0 / ((double)b.n3 * (double)b.n3);
    // block partials, then the per-shell second moments, in the rhs buffer (at least 20
    // bytes per point)
    const size_t room = b.n3 * 20 - (size_t)nshell * sizeof(double);
    const size_t cap = room / (2 * sizeof(double) * (size_t)nshell);
    const unsigned nb = (unsigned)std::max<size_t>(1, std::min<size_t>({cap, (size_t)1024, (size_t)pg}));
    double *part = (double *)b.rhs;
    double *M2 = part + (size_t)nb * 2 * nshell;
    const size_t hist = 2 * sizeof(double) * (size_t)nshell;
    hipLaunchKernelGGL(k_spec_bin, dim3(nb), dim3(kPointThreads), hist, s, X1, X2, G, part);
    hipLaunchKernelGGL(k_spec_final, dim3((unsigned)nshell), dim3(kPointThreads), 0, s, part, (int)nb, nshell, E, M2);
    hipLaunchKernelGGL(k_spec_mom, dim3(1), dim3(64), 0, s, E, M2, nshell, mom);
}

}  // namespace cns
