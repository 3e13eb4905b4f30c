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
//   3. binning: per-wave shell histograms in LDS, each run of equal shells in a wave
//      summed by a segmented scan and added by one lane at a time, then fixed-order
//      sums over the waves of a block, over blocks (one block per shell) and over
//      shells: the result is the same bits on every run.
// Scratch: the plan's stage buffers A (X1), B (X2) and rhs (block partials).
#include <cmath>
#include <vector>

#include "cns_internal.h"

namespace cns {

constexpr int kFftThreads = 256;
constexpr int kFftPerThread = 8;                           // elements a thread holds through a stage
constexpr int kFftElems = kFftThreads * kFftPerThread;     // nl * N per block
constexpr int kFftMaxRadix = 32;
constexpr size_t kFftLdsMax = 64 * 1024;
constexpr size_t kFftLineLds = 32 * 1024;                  // LDS for the lines of one block

// Exact unsigned division by a divisor fixed at launch: q = (umulhi(n, M) + n) >> l with
// l = ceil(log2 d) and M = floor(2^32 (2^l - d) / d) + 1 (the round-up multiply-shift of
// Granlund and Montgomery), exact for every 32-bit n.
struct FastDiv {
    uint32_t M;
    int l;
};
static FastDiv fastdiv(uint32_t d) {
    int l = 0;
    while ((1ull << l) < d) ++l;
    return FastDiv{(uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1), l};
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) {
    return (uint32_t)(((uint64_t)__umulhi(n, f.M) + n) >> f.l);
}
// Division of small numbers: with M = ceil(2^32 / d), floor(n M / 2^32) = floor(n / d)
// whenever n < 2^16 and d < 2^16 (the error n (M d - 2^32) / (d 2^32) stays below 1/d).
// The in-line indexes of the stages (below 2^13) use it, with M formed on the device.
__device__ __forceinline__ uint64_t small_magic(uint32_t d) { return (uint64_t)(0xFFFFFFFFu / d) + 1u; }
__device__ __forceinline__ int sdiv(int n, uint64_t M) { return (int)(((uint64_t)(uint32_t)n * M) >> 32); }

struct FftPlan {
    int N;            // line length
    int nr;           // number of radix stages
    int radix[kFftMaxRadix];
    FastDiv dN, dnl, dna;
    int nlines;
    int nl;           // lines per block (nl * N <= kFftElems)
    int ld;           // LDS stride between lines
    int swz;          // 14: XOR swizzle of the in-line index (N % 16 == 0, ld = N); 0: ld = N + 1
    int na;           // line index L -> (L % na) * sa + (L / na) * sb
    size_t sa, sb, es;
    int contig;       // 1: elements of a line are contiguous (x pass)
    const double2 *tw;  // tw[k] = exp(-2 pi i k / N), k < N (global; each block copies it to LDS)
};

// LDS slot of element j of line l.  Lines of the y and z passes are loaded with l
// fastest; the swizzle (or the padding) puts the lines of one index j in different banks.
__device__ __forceinline__ int lds_at(int l, int j, const FftPlan &P) {
    return l * P.ld + (j ^ ((l << 1) & P.swz));
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// One Stockham stage of radix R on nl lines of length N, in place in LDS: every thread
// reads the inputs of its butterflies into registers, the block synchronises, then the
// outputs are written.  Butterfly j (0 <= j < N/R) reads x[j + r N/R], r = 0..R-1,
// multiplies by the twiddles exp(-2 pi i r k/(Ns R)) with k = j mod Ns, takes a length-R
// DFT and writes output s to x[(j/Ns) Ns R + k + s Ns].
template <int R>
__device__ __forceinline__ void fft_stage_small(double2 *x, const double2 *tw, const FftPlan &P, int nl, int Ns) {
    const int N = P.N, m = N / R, tws = N / (Ns * R), nb = nl * m, tR = N / R;
    const uint64_t Mm = small_magic(m), Mns = small_magic(Ns);
    constexpr int NB = (kFftPerThread + R - 1) / R;
    double2 v[NB][R];
    int lo[NB], oo[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int t = threadIdx.x + q * kFftThreads;
        if (t < nb) {
            const int l = sdiv(t, Mm), j = t - l * m;
            const int jn = sdiv(j, Mns), k = j - jn * Ns;
            lo[q] = l;
            oo[q] = jn * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                v[q][r] = x[lds_at(l, j + r * m, P)];
                if (r) v[q][r] = cmul(v[q][r], tw[r * k * tws]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int t = threadIdx.x + q * kFftThreads;
        if (t < nb) {
            const int l = lo[q], o = oo[q];
            if constexpr (R == 2) {
                x[lds_at(l, o, P)] = cadd(v[q][0], v[q][1]);
                x[lds_at(l, o + Ns, P)] = csub(v[q][0], v[q][1]);
            } else if constexpr (R == 4) {
                const double2 s0 = cadd(v[q][0], v[q][2]), d0 = csub(v[q][0], v[q][2]);
                const double2 s1 = cadd(v[q][1], v[q][3]), d1 = csub(v[q][1], v[q][3]);
                const double2 md1 = make_double2(d1.y, -d1.x);  // -i * d1
                x[lds_at(l, o, P)] = cadd(s0, s1);
                x[lds_at(l, o + Ns, P)] = cadd(d0, md1);
                x[lds_at(l, o + 2 * Ns, P)] = csub(s0, s1);
                x[lds_at(l, o + 3 * Ns, P)] = csub(d0, md1);
            } else {
#pragma unroll
                for (int s = 0; s < R; ++s) {
                    double2 acc = v[q][0];
#pragma unroll
                    for (int r = 1; r < R; ++r) acc = cadd(acc, cmul(v[q][r], tw[((r * s) % R) * tR]));
                    x[lds_at(l, o + s * Ns, P)] = acc;
                }
            }
        }
    }
    __syncthreads();
}

// generic radix R (any prime above 5): one work item per output, outputs held in
// registers until every input has been read
__device__ __forceinline__ void fft_stage_generic(double2 *x, const double2 *tw, const FftPlan &P, int nl, int Ns,
                                                  int R) {
    const int N = P.N, m = N / R, tws = N / (Ns * R), tR = N / R;
    const uint64_t MN = small_magic(N), Mm = small_magic(m), Mns = small_magic(Ns);
    double2 out[kFftPerThread];
    int at[kFftPerThread];
#pragma unroll
    for (int q = 0; q < kFftPerThread; ++q) {
        const int t = threadIdx.x + q * kFftThreads;
        if (t < nl * N) {
            const int l = sdiv(t, MN), qq = t - l * N;
            const int s = sdiv(qq, Mm), j = qq - s * m;
            const int jn = sdiv(j, Mns), k = j - jn * Ns;
            double2 acc = x[lds_at(l, j, P)];
            int rs = 0;
            for (int r = 1; r < R; ++r) {
                rs += s;
                if (rs >= R) rs -= R;
                const double2 w = cmul(x[lds_at(l, j + r * m, P)], tw[r * k * tws]);
                acc = cadd(acc, cmul(w, tw[rs * tR]));
            }
            out[q] = acc;
            at[q] = lds_at(l, jn * Ns * R + k + s * Ns, P);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kFftPerThread; ++q) {
        const int t = threadIdx.x + q * kFftThreads;
        if (t < nl * N) x[at[q]] = out[q];
    }
    __syncthreads();
}

// Element offset of element j of line L in the field.
__device__ __forceinline__ size_t line_elem(const FftPlan &P, int L, int j) {
    const int hi = (int)fdiv(L, P.dna), lo = L - hi * P.na;
    return (size_t)lo * P.sa + (size_t)hi * P.sb + (size_t)j * P.es;
}

// Line and element of slot t of a block's line group (x pass: elements of one line are
// consecutive in t; y and z passes: lines are, so loads and stores coalesce along x).
__device__ __forceinline__ void slot_lj(const FftPlan &P, int t, int &l, int &j) {
    if (P.contig) {
        l = (int)fdiv(t, P.dN);
        j = t - l * P.N;
    } else {
        j = (int)fdiv(t, P.dnl);
        l = t - j * P.nl;
    }
}

// The thread index behind an empty asm: the slot indexes of the store phase are formed
// again instead of being kept live through the stages.
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Load the elements of the thread's slots of line group g into val (zero past the last
// line).
template <int SRC, typename T>
__device__ __forceinline__ void load_group(const FftPlan &P, const double2 *X, const T *u, size_t n3, int g,
                                           double2 (&val)[kFftPerThread]) {
    const int nl = P.nl, ne = nl * P.N;
    const int L0 = g * nl, nact = min(nl, P.nlines - L0);
    const int tid = opaque_tid();
#pragma unroll
    for (int q = 0; q < kFftPerThread; ++q) {
        const int t = tid + q * kFftThreads;
        val[q] = make_double2(0.0, 0.0);
        int l, j;
        slot_lj(P, t, l, j);
        if (t < ne && l < nact) {
            const size_t e = line_elem(P, L0 + l, j);
            if constexpr (SRC == 0) {
                val[q] = X[e];
            } else {
                const double r = double(u[e]);
                if constexpr (SRC == 1)
                    val[q] = make_double2(double(u[n3 + e]) / r, double(u[2 * n3 + e]) / r);
                else
                    val[q] = make_double2(double(u[3 * n3 + e]) / r, 0.0);
            }
        }
    }
}

// Batched 1-D FFTs of one pass.  SRC = 0: the lines of X are transformed in place.
// SRC = 1 or 2 (x pass only): the lines are formed from the state u, v_x + i v_y (1) or
// v_z (2), with v = m / rho, and the transform is written to X.  POW2: the line length is
// a power of two, so only the radix-4 and radix-2 stages are compiled in (104-120
// VGPRs instead of the 180-195 that the odd radices bring).  One line group per block.
template <int SRC, typename T, bool POW2>
__global__ __launch_bounds__(kFftThreads) void k_fft_lines(double2 *X, const T *u, size_t n3, FftPlan P) {
    extern __shared__ double2 lds_c[];  // [N] twiddles, then [nl][ld] lines
    double2 *tws = lds_c, *lines = lds_c + P.N;
    const int nl = P.nl;
    const int ne = nl * P.N;
    const int ngroups = (P.nlines + nl - 1) / nl;
    for (int k = threadIdx.x; k < P.N; k += kFftThreads) tws[k] = P.tw[k];
    for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int L0 = g * nl;
        const int nact = min(nl, P.nlines - L0);
        {
            double2 val[kFftPerThread];
            load_group<SRC, T>(P, X, u, n3, g, val);
            const int tid = opaque_tid();
#pragma unroll
            for (int q = 0; q < kFftPerThread; ++q) {
                const int t = tid + q * kFftThreads;
                int l, j;
                slot_lj(P, t, l, j);
                if (t < ne) lines[lds_at(l, j, P)] = val[q];
            }
        }
        __syncthreads();
        int Ns = 1;
        for (int st = 0; st < P.nr; ++st) {
            const int R = P.radix[st];
            if (R == 4) {
                fft_stage_small<4>(lines, tws, P, nl, Ns);
            } else if (R == 2) {
                fft_stage_small<2>(lines, tws, P, nl, Ns);
            } else if constexpr (!POW2) {
                if (R == 3) fft_stage_small<3>(lines, tws, P, nl, Ns);
                else if (R == 5) fft_stage_small<5>(lines, tws, P, nl, Ns);
                else fft_stage_generic(lines, tws, P, nl, Ns, R);
            }
            Ns *= R;
        }
        const int tid = opaque_tid();
#pragma unroll
        for (int q = 0; q < kFftPerThread; ++q) {
            const int t = tid + q * kFftThreads;
            int l, j;
            slot_lj(P, t, l, j);
            if (t < ne && l < nact) X[line_elem(P, L0 + l, j)] = lines[lds_at(l, j, P)];
        }
        __syncthreads();  // the next group reuses the LDS
    }
}

// tw[k] = exp(-2 pi i k / N), k < N
__global__ void k_fft_twiddles(double2 *tw, int N) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
        double s, c;
        sincospi(-2.0 * (double)k / (double)N, &s, &c);
        tw[k] = make_double2(c, s);
    }
}

struct SpecGeom {
    int nx, ny, nz, nshell;
    size_t n3;
    double kux, kuy, kuz;  // 2 pi / L_d
    double norm;           // 1 / n3^2
};

__device__ __forceinline__ int signed_freq(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

// Shell sums of one block in a fixed order.  Each wave keeps its own histogram in LDS.
// The lanes of a wave hold consecutive points, so equal shells come in runs of
// neighbouring lanes: a segmented scan (fixed doubling order) sums each run into its
// last lane, and those lanes add to the histogram one at a time, in lane order (an add
// issued by a single lane has no partner to race with, and a wave's LDS operations
// complete in program order).  The wave histograms are summed in wave order at the
// end.  Every sum is thus formed in the same order on every run.
// Blocks of two waves, or of one where two histograms would pass 64 KiB of LDS.
// Up to 8192 blocks: the loop of a wave is latency bound (loads, the scan's lane
// exchanges, the ordered adds), so it needs many waves in flight.
constexpr int kSpecBinThreads = 128;
constexpr size_t kSpecBinLds = 64 * 1024;
constexpr size_t kSpecBinBlocksMax = 8192;
__global__ __launch_bounds__(kSpecBinThreads) void k_spec_bin(const double2 *X1, const double2 *X2, SpecGeom G,
                                                              double *part) {
    extern __shared__ double hist[];  // [wave][2][nshell]: E, |k|^2 E
    const int ns2 = 2 * G.nshell, waves = (int)blockDim.x >> 6;
    for (int s = threadIdx.x; s < waves * ns2; s += blockDim.x) hist[s] = 0.0;
    __syncthreads();
    const int lane = (int)threadIdx.x & 63;
    double *hw = hist + (size_t)(threadIdx.x >> 6) * ns2;
    // every lane of a wave runs the same number of rounds (lanes past the end add nothing)
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t first = blockIdx.x * (size_t)blockDim.x + (threadIdx.x & ~63u);
    for (size_t i0 = first; i0 < G.n3; i0 += stride) {
        const size_t i = i0 + lane;
        int s = -1;  // no shell: a run of its own that adds nothing
        double p = 0.0, q = 0.0;
        if (i < G.n3) {
            const int ix = (int)(i % G.nx);
            const int iy = (int)((i / G.nx) % G.ny);
            const int iz = (int)(i / ((size_t)G.nx * G.ny));
            const double kx = signed_freq(ix, G.nx) * G.kux, ky = signed_freq(iy, G.ny) * G.kuy,
                         kz = signed_freq(iz, G.nz) * G.kuz;
            const double k2 = kx * kx + ky * ky + kz * kz;
            s = min((int)floor(sqrt(k2) + 0.5), G.nshell - 1);
            const double2 a = X1[i], b = X2[i];
            p = 0.5 * (a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y) * G.norm;
            q = k2 * p;
        }
        // run heads and tails
        const int sp = __shfl_up(s, 1, 64), sn = __shfl_down(s, 1, 64);
        int f = (lane == 0 || sp != s) ? 1 : 0;
        const bool tail = lane == 63 || sn != s;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double pu = __shfl_up(p, d, 64), qu = __shfl_up(q, d, 64);
            const int fu = __shfl_up(f, d, 64);
            if (lane >= d) {
                if (!f) {
                    p += pu;
                    q += qu;
                }
                f |= fu;
            }
        }
        unsigned long long m = __ballot(tail && s >= 0);
        while (m) {
            const int l = __ffsll(m) - 1;
            if (lane == l) {
                atomicAdd(&hw[s], p);
                atomicAdd(&hw[G.nshell + s], q);
            }
            m &= m - 1;
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < ns2; s += blockDim.x) {
        double a = hist[s];
        for (int w = 1; w < waves; ++w) a += hist[(size_t)w * ns2 + s];
        part[(size_t)blockIdx.x * ns2 + s] = a;
    }
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

// mom = {sum_s E[s], sum_s M2[s]} in shell order, and the Taylor microscale
// lambda = sqrt(5 sum E / M2) of isotropic turbulence (+inf for a uniform velocity)
__global__ void k_spec_mom(const double *E, const double *M2, int nshell, double *mom) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double e = 0.0, m = 0.0;
    for (int s = 0; s < nshell; ++s) {
        e += E[s];
        m += M2[s];
    }
    mom[0] = e;
    mom[1] = m;
    mom[2] = m > 0.0 ? sqrt(5.0 * e / m) : __builtin_inf();
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
        if (n[d] > 2047) return false;
    // the shell histogram must fit in LDS, one block's partials and the per-shell second
    // moments in the rhs buffer (at least 20 bytes per point)
    const size_t hist = 2 * sizeof(double) * (size_t)spectrum_shells(b);
    return hist <= kFftLdsMax && hist + sizeof(double) * (size_t)spectrum_shells(b) <= 20 * b.n3;
}

// One pass of batched line FFTs along direction dir.  SRC as in k_fft_lines; tw holds the
// twiddle table of this direction's length.
template <int SRC, typename T>
static void fft_pass(double2 *X, const T *u, const BoxDesc &b, int dir, const double2 *tw, hipStream_t s) {
    FftPlan P{};
    const size_t nx = b.nx, ny = b.ny;
    P.N = dir == 0 ? b.nx : (dir == 1 ? b.ny : b.nz);
    P.nr = fft_factor(P.N, P.radix);
    P.nlines = (int)(b.n3 / P.N);
    if (dir == 0) {
        P.na = P.nlines, P.sa = nx, P.sb = 0, P.es = 1, P.contig = 1;
    } else if (dir == 1) {
        P.na = (int)nx, P.sa = 1, P.sb = nx * ny, P.es = nx, P.contig = 0;
    } else {
        P.na = P.nlines, P.sa = 1, P.sb = 0, P.es = nx * ny, P.contig = 0;
    }
    // lines per block: at most kFftElems elements and the line LDS budget, at most 64 lines
    P.swz = P.N % 16 == 0 ? 14 : 0;
    P.ld = P.swz ? P.N : P.N + 1;
    const int nl = std::max(1, std::min({64, kFftElems / P.N, (int)(kFftLineLds / (sizeof(double2) * P.ld))}));
    P.nl = nl;
    P.dN = fastdiv((uint32_t)P.N);
    P.dnl = fastdiv((uint32_t)nl);
    P.dna = fastdiv((uint32_t)P.na);
    P.tw = tw;
    const size_t lds = sizeof(double2) * ((size_t)nl * P.ld + P.N);
    const long long groups = (P.nlines + nl - 1) / nl;
    const unsigned grid = (unsigned)std::min<long long>(groups, 1 << 20);
    if ((P.N & (P.N - 1)) == 0)
        hipLaunchKernelGGL((k_fft_lines<SRC, T, true>), dim3(grid), dim3(kFftThreads), lds, s, X, u, b.n3, P);
    else
        hipLaunchKernelGGL((k_fft_lines<SRC, T, false>), dim3(grid), dim3(kFftThreads), lds, s, X, u, b.n3, P);
}

template <typename T>
static void spectrum_transforms(const BoxDesc &b, hipStream_t s, const T *u, double2 *X1, double2 *X2,
                                double2 *tw) {
    // twiddle tables of the three lengths at the start of the rhs buffer (free until the
    // binning below writes its partials there)
    const int n[3] = {b.nx, b.ny, b.nz};
    const double2 *twd[3];
    double2 *t = tw;
    for (int d = 0; d < 3; ++d) {
        hipLaunchKernelGGL(k_fft_twiddles, dim3((n[d] + 255) / 256), dim3(256), 0, s, t, n[d]);
        twd[d] = t;
        t += n[d];
    }
    fft_pass<1, T>(X1, u, b, 0, twd[0], s);
    fft_pass<2, T>(X2, u, b, 0, twd[0], s);
    for (int d = 1; d < 3; ++d) {
        fft_pass<0, T>(X1, nullptr, b, d, twd[d], s);
        fft_pass<0, T>(X2, nullptr, b, d, twd[d], s);
    }
}

void launch_spectrum(const BoxDesc &b, int prec, hipStream_t s, const void *u, double *E, int nshell, double *mom) {
    double2 *X1 = (double2 *)b.A, *X2 = (double2 *)b.B;
    const unsigned pg = (unsigned)std::min<size_t>((b.n3 + kSpecBinThreads - 1) / kSpecBinThreads, 65536);
    if (prec == CNS_FP64)
        spectrum_transforms<double>(b, s, (const double *)u, X1, X2, (double2 *)b.rhs);
    else
        spectrum_transforms<float>(b, s, (const float *)u, X1, X2, (double2 *)b.rhs);
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
    const unsigned nb = (unsigned)std::max<size_t>(1, std::min<size_t>({cap, (size_t)kSpecBinBlocksMax, (size_t)pg}));
    double *part = (double *)b.rhs;
    double *M2 = part + (size_t)nb * 2 * nshell;
    const size_t hist1 = 2 * sizeof(double) * (size_t)nshell;  // one wave's histogram
    const int waves = 2 * hist1 <= kSpecBinLds ? 2 : 1;
    hipLaunchKernelGGL(k_spec_bin, dim3(nb), dim3(64 * waves), waves * hist1, s, X1, X2, G, part);
    hipLaunchKernelGGL(k_spec_final, dim3((unsigned)nshell), dim3(kPointThreads), 0, s, part, (int)nb, nshell, E, M2);
    hipLaunchKernelGGL(k_spec_mom, dim3(1), dim3(64), 0, s, E, M2, nshell, mom);
}

}  // namespace cns
