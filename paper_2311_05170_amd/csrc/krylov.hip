// Matrix-free Krylov solver of the local Oseen systems (Eq. (5.8) on each
// Omega_cj) for boxes too wide for the band factorisation: restarted
// flexible GMRES in FP64, one workgroup per system for the Arnoldi vector
// work (uneven system sizes in one launch), preconditioned by restricted
// additive Schwarz over strips of the box.  The operator is applied by the
// FP64 tiled residual kernel (r = -K z); the strip systems are banded and
// solved by the band kernels with factors of the precision of the run.
//
// Every kernel skips a system whose `done` flag is set, so a fixed sequence
// of launches serves systems that converge after different iteration counts.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace lp {

namespace {

constexpr int GT = 512;                 // threads per system workgroup
constexpr int GW = GT / 64;

__device__ __forceinline__ double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sum of v over the workgroup, the same on every thread (fixed order: lanes by
// butterfly, then wavefronts in index order); red holds GW doubles
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wsum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < GW; ++i) s += red[i];
    return s;
}

}  // namespace

// beta = ||r||, ||b||, v_0 = r / beta, g = (beta, 0, ...), per system
__global__ __launch_bounds__(GT) void k_gm_init(GmresArgs G, const double *r, const double *b, int first) {
    const int s = blockIdx.x;
    const SysDesc S = G.sys[s];
    __shared__ double red[GW];
    const int n = S.ndof;
    if (first && threadIdx.x == 0) G.tot[s] = 0;
    if (G.conv && G.conv[s]) {
        if (threadIdx.x == 0) { G.done[s] = 1; G.kdone[s] = 0; }
        return;
    }
    const double *rs = r + S.dof_off, *bs = b + S.dof_off;
    double rr = 0.0, bb = 0.0;
    for (int i = threadIdx.x; i < n; i += GT) { rr += rs[i] * rs[i]; bb += bs[i] * bs[i]; }
    const double beta = sqrt(block_sum(rr, red));
    const double bn = sqrt(block_sum(bb, red));
    const bool stop = !(beta > G.tol * bn) || !(beta > 0.0);
    double *v0 = G.V + S.dof_off;
    const double sc = stop ? 0.0 : 1.0 / beta;
    for (int i = threadIdx.x; i < n; i += GT) v0[i] = rs[i] * sc;
    if (threadIdx.x == 0) {
        double *g = G.g + (long long)s * (G.m + 1);
        g[0] = beta;
        for (int i = 1; i <= G.m; ++i) g[i] = 0.0;
        G.bnorm[s] = bn;
        G.done[s] = stop ? 1 : 0;
        G.kdone[s] = 0;
    }
}

// Arnoldi step k: w = -wneg (= K z_k), h_i = <w, v_i> (i <= k, classical
// Gram-Schmidt against the stored basis), w -= sum h_i v_i, v_{k+1} = w / ||w||,
// then the Givens rotations of the Hessenberg column and the residual
// estimate |g_{k+1}|.  w is staged in LDS (dynamic, max ndof doubles).
__global__ __launch_bounds__(GT) void k_gm_arnoldi(GmresArgs G, int k, const double *wneg) {
    const int s = blockIdx.x;
    if (G.done[s]) return;
    const SysDesc S = G.sys[s];
    extern __shared__ double wl[];
    __shared__ double red[GW];
    __shared__ double hcol[GM_MAX + 1];
    const int n = S.ndof;
    const long long off = S.dof_off, nt = G.ntot;
    const double *ws = wneg + off;
    for (int i = threadIdx.x; i < n; i += GT) wl[i] = -ws[i];
    __syncthreads();
    for (int j = 0; j <= k; ++j) {
        const double *vj = G.V + j * nt + off;
        double p = 0.0;
        for (int i = threadIdx.x; i < n; i += GT) p += wl[i] * vj[i];
        p = block_sum(p, red);
        if (threadIdx.x == 0) hcol[j] = p;
    }
    __syncthreads();
    double nn = 0.0;
    for (int i = threadIdx.x; i < n; i += GT) {
        double a = wl[i];
        for (int j = 0; j <= k; ++j) a -= hcol[j] * G.V[j * nt + off + i];
        wl[i] = a;
        nn += a * a;
    }
    if (G.reorth) {
        // a second Gram-Schmidt pass against the same basis (its coefficients
        // added to the Hessenberg column)
        __shared__ double h2[GM_MAX + 1];
        for (int j = 0; j <= k; ++j) {
            const double *vj = G.V + j * nt + off;
            double p = 0.0;
            for (int i = threadIdx.x; i < n; i += GT) p += wl[i] * vj[i];
            p = block_sum(p, red);
            if (threadIdx.x == 0) h2[j] = p;
        }
        __syncthreads();
        nn = 0.0;
        for (int i = threadIdx.x; i < n; i += GT) {
            double a = wl[i];
            for (int j = 0; j <= k; ++j) a -= h2[j] * G.V[j * nt + off + i];
            wl[i] = a;
            nn += a * a;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int j = 0; j <= k; ++j) hcol[j] += h2[j];
    }
    const double nrm = sqrt(block_sum(nn, red));
    const double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
    double *vk1 = G.V + (k + 1) * nt + off;
    for (int i = threadIdx.x; i < n; i += GT) vk1[i] = wl[i] * sc;
    if (threadIdx.x == 0) {
        const int m = G.m;
        double *H = G.H + (long long)s * (m + 1) * m + (long long)k * (m + 1);
        double *cs = G.cs + (long long)s * m, *sn = G.sn + (long long)s * m;
        double *g = G.g + (long long)s * (m + 1);
        hcol[k + 1] = nrm;
        for (int j = 0; j < k; ++j) {
            const double a = hcol[j], b = hcol[j + 1];
            hcol[j] = cs[j] * a + sn[j] * b;
            hcol[j + 1] = -sn[j] * a + cs[j] * b;
        }
        const double a = hcol[k], b = hcol[k + 1];
        const double rr = sqrt(a * a + b * b);
        const double c = rr > 0.0 ? a / rr : 1.0, sg = rr > 0.0 ? b / rr : 0.0;
        cs[k] = c;
        sn[k] = sg;
        hcol[k] = rr;
        hcol[k + 1] = 0.0;
        g[k + 1] = -sg * g[k];
        g[k] = c * g[k];
        for (int j = 0; j <= k + 1; ++j) H[j] = hcol[j];
        G.kdone[s] = k + 1;
        const bool conv = fabs(g[k + 1]) <= G.tol * G.bnorm[s];
        if (conv || k + 1 >= m || !(nrm > 0.0) || !(rr > 0.0)) G.done[s] = 1;
    }
}

// x += Z y with R y = g (R the rotated Hessenberg of the steps taken)
__global__ __launch_bounds__(GT) void k_gm_update(GmresArgs G, double *x) {
    const int s = blockIdx.x;
    const int kd = G.kdone[s];
    if (kd <= 0) return;
    const SysDesc S = G.sys[s];
    __shared__ double y[GM_MAX];
    const int m = G.m;
    if (threadIdx.x == 0) {
        const double *H = G.H + (long long)s * (m + 1) * m;
        const double *g = G.g + (long long)s * (m + 1);
        for (int i = kd - 1; i >= 0; --i) {
            double a = g[i];
            for (int j = i + 1; j < kd; ++j) a -= H[(long long)j * (m + 1) + i] * y[j];
            const double d = H[(long long)i * (m + 1) + i];
            y[i] = d != 0.0 ? a / d : 0.0;
        }
    }
    if (threadIdx.x == 0) G.tot[s] += kd;
    __syncthreads();
    const int n = S.ndof;
    const long long off = S.dof_off, nt = G.ntot;
    for (int i = threadIdx.x; i < n; i += GT) {
        double a = x[off + i];
        for (int j = 0; j < kd; ++j) a += y[j] * G.Z[j * nt + off + i];
        x[off + i] = a;
    }
}

// strip right-hand sides from the parent vector v (one workgroup per strip);
// strips of finished systems are flagged for the band solve to skip
__global__ __launch_bounds__(256) void k_strip_gather(StripArgs A, const double *v) {
    const int st = blockIdx.x;
    const SysDesc S = A.strip[st];
    const int par = A.parent[st];
    const int skip = A.done[par];
    if (threadIdx.x == 0) A.sdone[st] = skip;
    if (skip) return;
    const long long po = A.sys[par].dof_off;
    for (int i = threadIdx.x; i < S.ndof; i += blockDim.x)
        A.rs[S.dof_off + i] = v[po + A.smap[S.dof_off + i]];
}

// z_k on the parent unknowns owned by each strip (restricted additive Schwarz)
__global__ __launch_bounds__(256) void k_strip_scatter(StripArgs A, double *z) {
    const int st = blockIdx.x;
    const SysDesc S = A.strip[st];
    const int par = A.parent[st];
    if (A.done[par]) return;
    const long long po = A.sys[par].dof_off;
    for (int i = threadIdx.x; i < S.ndof; i += blockDim.x)
        if (A.sown[S.dof_off + i]) z[po + A.smap[S.dof_off + i]] = A.zs[S.dof_off + i];
}

// a smooth fixed vector (autotuning right-hand sides): x_i = sin(0.37 i) + 0.5
__global__ void k_fill_pattern(double *x, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] = sin(0.37 * (double)i) + 0.5;
}

size_t gm_arnoldi_lds(int maxn) { return (size_t)maxn * sizeof(double); }

void launch_fill_pattern(double *x, long long n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_pattern, dim3((unsigned)std::min<long long>(1024, (n + 255) / 256)), dim3(256), 0, st, x, n);
}

bool launch_gm_init(const GmresArgs &a, int nsys, const double *r, const double *b, bool first, hipStream_t st) {
    hipLaunchKernelGGL(k_gm_init, dim3(nsys), dim3(GT), 0, st, a, r, b, first ? 1 : 0);
    return true;
}
bool launch_gm_arnoldi(const GmresArgs &a, int nsys, int maxn, int k, const double *wneg, hipStream_t st) {
    const size_t sh = gm_arnoldi_lds(maxn);
    if (sh > GM_LDS_MAX || k < 0 || k >= a.m || a.m > GM_MAX) return false;
    hipLaunchKernelGGL(k_gm_arnoldi, dim3(nsys), dim3(GT), sh, st, a, k, wneg);
    return true;
}
void launch_gm_update(const GmresArgs &a, int nsys, double *x, hipStream_t st) {
    hipLaunchKernelGGL(k_gm_update, dim3(nsys), dim3(GT), 0, st, a, x);
}
void launch_strip_gather(const StripArgs &a, int nstrip, const double *v, hipStream_t st) {
    hipLaunchKernelGGL(k_strip_gather, dim3(nstrip), dim3(256), 0, st, a, v);
}
void launch_strip_scatter(const StripArgs &a, int nstrip, double *z, hipStream_t st) {
    hipLaunchKernelGGL(k_strip_scatter, dim3(nstrip), dim3(256), 0, st, a, z);
}

}  // namespace lp
