/*
 * kernels_krylov.hip -- the alternative CG methods of Sec. 4.1 on the GPU,
 * without preconditioner as the paper compares them.  Both use the
 * operator's plain mat-vec mode (fused tile kernel + shared-node kernel)
 * and loop-fused streaming vector kernels around it:
 *
 *  Pipelined CG (Algorithm 2).  The scalars of iteration k depend only on
 *  the two inner products of iteration k-1, so after q = A w one kernel
 *  applies all six vector updates (p, x, s, r, z, w) and forms the partial
 *  sums of gamma = r^T r and a = w^T r: 7 vectors read, 6 written.  As the
 *  paper suggests, x takes two steps at once every other iteration
 *  (x += alpha_{k-1} p_{k-1} + alpha_k p_k, with p_{k-1} read before its
 *  update), 6.5 reads and 5.5 writes on average; an odd exit owes x one
 *  step, added at the end.  A one-block finish turns the inner products
 *  into the next alpha and beta.
 *
 *  s-step CG (Algorithm 3, monomial basis).  Per phase of s iterations the
 *  caller runs the s mat-vecs of the basis T = [r, A r, .., A^s r], then
 *    pass 1: C = P_prev^T Q                       (2s vectors read)
 *    pass 2: P = R + P_prev B, W = Q^T P, g = P^T r (2s+1 read, s written)
 *    pass 3: x += P a                             (s+1 read, 1 written)
 *  and, after the mat-vec v = A x,
 *    pass 4: r = b - v, gamma = r^T r              (2 read, 1 written)
 *  where R = T[0..s), Q = T[1..s], B = -W_prev^{-1} C and a = W^{-1} g
 *  come from s x s solves (Gaussian elimination with partial pivoting) done
 *  by one thread between the passes.  The first phase takes P = R.
 *
 * All reductions write per-block records that one block adds in a fixed
 * order, so runs are reproducible.  Every kernel returns at once when the
 * solve has stopped (converged, broken down).
 */
#include <hip/hip_runtime.h>

#include "cg_common.h"
#include "kernels.h"

namespace mfcg {

constexpr int KV_WG = 256; /* the block size vec_blocks() sizes grids for */

/* Fixed-order sums of NV values over nparts records of REC doubles.  The
 * block splits into SHARED_WG / NV groups of NV threads; thread c of group
 * g adds value c of records g, g + groups, ... (neighbouring threads read
 * neighbouring values of one record; eight records in flight per thread),
 * then one thread per value adds the groups' sums in group order.  red
 * holds SHARED_WG doubles. */
template <int NV, int REC>
__device__ void sum_records(const double *part, int64_t nparts, double *red, double *tot)
{
    static_assert(NV <= SHARED_WG, "one thread per value at least");
    constexpr int NG = SHARED_WG / NV;
    const int g = threadIdx.x / NV, c = threadIdx.x - g * NV;
    constexpr int U = 8; /* records in flight per thread */
    double acc = 0.0;
    if (g < NG)
        for (int64_t b0 = g; b0 < nparts; b0 += (int64_t)NG * U) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t b = b0 + (int64_t)u * NG;
                v[u] = b < nparts ? part[b * REC + c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc += v[u];
        }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
        for (int gg = 0; gg < NG; ++gg) t += red[gg * NV + threadIdx.x];
        tot[threadIdx.x] = t;
    }
    __syncthreads();
}

/* ---------------- pipelined CG ---------------- */

__global__ __launch_bounds__(KV_WG) void pipe_init_kernel(const PipeArgs a)
{
    __shared__ double red[2 * (KV_WG / 64)];
    if (a.st->flag != FLAG_RUN) return;
    double acc[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * KV_WG;
    for (int64_t i = (int64_t)blockIdx.x * KV_WG + threadIdx.x; i < a.n; i += stride) {
        const double r = a.r[i], w = a.w[i];
        a.p[i] = 0.0;
        a.s[i] = 0.0;
        a.z[i] = 0.0;
        acc[0] += r * r;
        acc[1] += w * r;
    }
    block_reduce<double, 2, KV_WG>(acc, red, a.part + (int64_t)blockIdx.x * 8);
}

__global__ __launch_bounds__(KV_WG) void pipe_vec_kernel(const PipeArgs a)
{
    __shared__ double red[2 * (KV_WG / 64)];
    if (a.st->flag != FLAG_RUN) return;
    const double alpha = a.ks->alpha, beta = a.ks->beta, alpha_prev = a.ks->alpha_prev;
    const bool xupd = ((a.st->k + 1) & 1) == 0; /* even iterations update x */
    double acc[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * KV_WG;
    for (int64_t i = (int64_t)blockIdx.x * KV_WG + threadIdx.x; i < a.n; i += stride) {
        const double r = a.r[i], w = a.w[i], q = a.q[i], pold = a.p[i];
        const double p = fma(beta, pold, r);
        const double sv = fma(beta, a.s[i], w);
        const double z = fma(beta, a.z[i], q);
        const double rn = fma(-alpha, sv, r);
        const double wn = fma(-alpha, z, w);
        if (xupd) a.x[i] = fma(alpha, p, fma(alpha_prev, pold, a.x[i]));
        a.p[i] = p;
        a.s[i] = sv;
        a.z[i] = z;
        a.r[i] = rn;
        a.w[i] = wn;
        acc[0] += rn * rn;
        acc[1] += wn * rn;
    }
    block_reduce<double, 2, KV_WG>(acc, red, a.part + (int64_t)blockIdx.x * 8);
}

/* INIT: gamma_0, a_0 -> alpha_1 (beta_1 = 0).  Otherwise gamma_k, a_k of
 * iteration k: history, convergence test on sqrt(gamma_k), then
 * beta_{k+1} = gamma_k / gamma_{k-1} and
 * alpha_{k+1} = gamma_k / (a_k - beta_{k+1} gamma_k / alpha_k). */
template <int INIT>
__global__ __launch_bounds__(SHARED_WG) void pipe_finish_kernel(const PipeArgs a, int64_t nparts)
{
    __shared__ double red[SHARED_WG];
    __shared__ double tot[2];
    CGState *st = a.st;
    if (st->flag != FLAG_RUN) return;
    sum_records<2, 8>(a.part, nparts, red, tot);
    if (threadIdx.x != 0) return;
    KrylovState *ks = a.ks;
    const double g = tot[0], wr = tot[1];
    if (INIT) ks->xpend = 0;
    if (!INIT) {
        const int k = st->k + 1;
        const double rho = sqrt(g);
        a.hist[k] = rho;
        st->k = k;
        ks->alpha_x = ks->alpha; /* the step of iteration k */
        ks->xpend = k & 1;
        if (!isfinite(g)) {
            st->flag = FLAG_BREAK;
            return;
        }
        if (rho < st->eps) {
            st->flag = FLAG_CONV;
            return;
        }
        if (k >= st->maxit) return; /* no next iteration to prepare */
    }
    const double beta = INIT ? 0.0 : g / ks->gamma;
    const double den = INIT ? wr : wr - beta * g / ks->alpha;
    if (!(den > 0) || !isfinite(den)) {
        st->flag = FLAG_BREAK; /* the next iteration cannot start */
        st->k += 1;
        return;
    }
    ks->alpha_prev = ks->alpha;
    ks->alpha = g / den;
    ks->beta = beta;
    ks->gamma = g;
    ks->a = wr;
}

/* exit: an odd iteration count leaves the last step alpha_k p_k owed to x */
__global__ __launch_bounds__(KV_WG) void pipe_exit_kernel(const PipeArgs a)
{
    if (!a.ks->xpend) return;
    const double alpha = a.ks->alpha_x;
    const int64_t stride = (int64_t)gridDim.x * KV_WG;
    for (int64_t i = (int64_t)blockIdx.x * KV_WG + threadIdx.x; i < a.n; i += stride) a.x[i] = fma(alpha, a.p[i], a.x[i]);
}

hipError_t launch_pipe_exit(const PipeArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(pipe_exit_kernel, dim3(vec_blocks(a.n)), dim3(KV_WG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pipe_init(const PipeArgs &a, hipStream_t s)
{
    const int nb = vec_blocks(a.n);
    hipLaunchKernelGGL(pipe_init_kernel, dim3(nb), dim3(KV_WG), 0, s, a);
    hipLaunchKernelGGL(pipe_finish_kernel<1>, dim3(1), dim3(SHARED_WG), 0, s, a, (int64_t)nb);
    return hipGetLastError();
}

hipError_t launch_pipe_step(const PipeArgs &a, hipStream_t s)
{
    const int nb = vec_blocks(a.n);
    hipLaunchKernelGGL(pipe_vec_kernel, dim3(nb), dim3(KV_WG), 0, s, a);
    hipLaunchKernelGGL(pipe_finish_kernel<0>, dim3(1), dim3(SHARED_WG), 0, s, a, (int64_t)nb);
    return hipGetLastError();
}

/* ---------------- s-step CG ---------------- */

/* Solves M X = Rh in place (X in Rh) by Gaussian elimination with partial
 * pivoting; false on a zero pivot or a non-finite result. */
template <int S, int NR>
__device__ bool gepp_solve(double (&M)[S][S], double (&Rh)[S][NR])
{
    for (int c = 0; c < S; ++c) {
        int piv = c;
        double best = fabs(M[c][c]);
        for (int r = c + 1; r < S; ++r)
            if (fabs(M[r][c]) > best) {
                best = fabs(M[r][c]);
                piv = r;
            }
        if (!(best > 0.0) || !isfinite(best)) return false;
        if (piv != c) {
            for (int j = 0; j < S; ++j) {
                const double t = M[c][j];
                M[c][j] = M[piv][j];
                M[piv][j] = t;
            }
            for (int j = 0; j < NR; ++j) {
                const double t = Rh[c][j];
                Rh[c][j] = Rh[piv][j];
                Rh[piv][j] = t;
            }
        }
        for (int r = c + 1; r < S; ++r) {
            const double f = M[r][c] / M[c][c];
            for (int j = c; j < S; ++j) M[r][j] -= f * M[c][j];
            for (int j = 0; j < NR; ++j) Rh[r][j] -= f * Rh[c][j];
        }
    }
    bool ok = true;
    for (int c = S - 1; c >= 0; --c)
        for (int j = 0; j < NR; ++j) {
            double t = Rh[c][j];
            for (int m = c + 1; m < S; ++m) t -= M[c][m] * Rh[m][j];
            t /= M[c][c];
            Rh[c][j] = t;
            ok = ok && isfinite(t);
        }
    return ok;
}

/* pass 1: C[m][l] = P_prev[m]^T Q[l], Q[l] = T[l+1] (skipped in the first phase) */
template <int S>
__global__ __launch_bounds__(KV_WG) void sstep_c_kernel(const SStepArgs a)
{
    __shared__ double red[S * S * (KV_WG / 64)];
    if (a.st->flag != FLAG_RUN || a.ks->phase == 0) return;
    double acc[S * S];
#pragma unroll
    for (int c = 0; c < S * S; ++c) acc[c] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * KV_WG;
    for (int64_t i = (int64_t)blockIdx.x * KV_WG + threadIdx.x; i < a.n; i += stride) {
        double pp[S], q[S];
#pragma unroll
        for (int m = 0; m < S; ++m) pp[m] = a.P[m][i];
#pragma unroll
        for (int l = 0; l < S; ++l) q[l] = a.T[l + 1][i];
#pragma unroll
        for (int m = 0; m < S; ++m)
#pragma unroll
            for (int l = 0; l < S; ++l) acc[m * S + l] = fma(pp[m], q[l], acc[m * S + l]);
    }
    block_reduce<double, S * S, KV_WG>(acc, red, a.part + (int64_t)blockIdx.x * SSTEP_REC);
}

/* B = -W_prev^{-1} C */
template <int S>
__global__ __launch_bounds__(SHARED_WG) void sstep_b_finish(const SStepArgs a, int64_t nparts)
{
    __shared__ double red[SHARED_WG];
    __shared__ double tot[S * S];
    CGState *st = a.st;
    KrylovState *ks = a.ks;
    if (st->flag != FLAG_RUN || ks->phase == 0) return;
    sum_records<S * S, SSTEP_REC>(a.part, nparts, red, tot);
    if (threadIdx.x != 0) return;
    double M[S][S], X[S][S];
    for (int m = 0; m < S; ++m)
        for (int l = 0; l < S; ++l) {
            M[m][l] = ks->W[m * S + l];
            X[m][l] = tot[m * S + l];
        }
    if (!gepp_solve<S, S>(M, X)) {
        st->flag = FLAG_BREAK;
        st->k += S;
        return;
    }
    for (int m = 0; m < S; ++m)
        for (int l = 0; l < S; ++l) ks->B[m * S + l] = -X[m][l];
}

/* pass 2: P[l] = T[l] + sum_m P_prev[m] B[m][l] (P = R in the first phase);
 * W[m][l] = Q[m]^T P[l]; g[l] = P[l]^T r */
template <int S>
__global__ __launch_bounds__(KV_WG) void sstep_p_kernel(const SStepArgs a)
{
    constexpr int NV = S * S + S;
    __shared__ double red[NV * (KV_WG / 64)];
    if (a.st->flag != FLAG_RUN) return;
    const bool prev = a.ks->phase > 0;
    double B[S * S];
#pragma unroll
    for (int c = 0; c < S * S; ++c) B[c] = prev ? a.ks->B[c] : 0.0;
    double acc[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[c] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * KV_WG;
    for (int64_t i = (int64_t)blockIdx.x * KV_WG + threadIdx.x; i < a.n; i += stride) {
        double t[S + 1], pn[S];
#pragma unroll
        for (int j = 0; j <= S; ++j) t[j] = a.T[j][i];
        if (prev) {
            double pp[S];
#pragma unroll
            for (int m = 0; m < S; ++m) pp[m] = a.P[m][i];
#pragma unroll
            for (int l = 0; l < S; ++l) {
                double u = 0.0;
#pragma unroll
                for (int m = 0; m < S; ++m) u = fma(pp[m], B[m * S + l], u);
                pn[l] = t[l] + u;
            }
        } else {
#pragma unroll
            for (int l = 0; l < S; ++l) pn[l] = t[l];
        }
#pragma unroll
        for (int l = 0; l < S; ++l) a.P[l][i] = pn[l];
#pragma unroll
        for (int m = 0; m < S; ++m)
#pragma unroll
            for (int l = 0; l < S; ++l) acc[m * S + l] = fma(t[m + 1], pn[l], acc[m * S + l]);
#pragma unroll
        for (int l = 0; l < S; ++l) acc[S * S + l] = fma(pn[l], t[0], acc[S * S + l]);
    }
    block_reduce<double, NV, KV_WG>(acc, red, a.part + (int64_t)blockIdx.x * SSTEP_REC);
}

/* keep W for the next phase; a = W^{-1} g */
template <int S>
__global__ __launch_bounds__(SHARED_WG) void sstep_a_finish(const SStepArgs a, int64_t nparts)
{
    constexpr int NV = S * S + S;
    __shared__ double red[SHARED_WG];
    __shared__ double tot[NV];
    CGState *st = a.st;
    KrylovState *ks = a.ks;
    if (st->flag != FLAG_RUN) return;
    sum_records<NV, SSTEP_REC>(a.part, nparts, red, tot);
    if (threadIdx.x != 0) return;
    double M[S][S], g[S][1];
    for (int m = 0; m < S; ++m) {
        for (int l = 0; l < S; ++l) {
            M[m][l] = tot[m * S + l];
            ks->W[m * S + l] = tot[m * S + l];
        }
        g[m][0] = tot[S * S + m];
    }
    if (!gepp_solve<S, 1>(M, g)) {
        st->flag = FLAG_BREAK;
        st->k += S;
        return;
    }
    for (int m = 0; m < S; ++m) ks->avec[m] = g[m][0];
}

/* pass 3: x += P a */
template <int S>
__global__ __launch_bounds__(KV_WG) void sstep_x_kernel(const SStepArgs a)
{
    if (a.st->flag != FLAG_RUN) return;
    double c[S];
#pragma unroll
    for (int l = 0; l < S; ++l) c[l] = a.ks->avec[l];
    const int64_t stride = (int64_t)gridDim.x * KV_WG;
    for (int64_t i = (int64_t)blockIdx.x * KV_WG + threadIdx.x; i < a.n; i += stride) {
        double u = 0.0;
#pragma unroll
        for (int l = 0; l < S; ++l) u = fma(a.P[l][i], c[l], u);
        a.x[i] += u;
    }
}

/* pass 4: r = T[0] = b - v, partial gamma */
__global__ __launch_bounds__(KV_WG) void sstep_r_kernel(const SStepArgs a)
{
    __shared__ double red[KV_WG / 64];
    if (a.st->flag != FLAG_RUN) return;
    double acc[1] = {0.0};
    double *r = a.T[0];
    const int64_t stride = (int64_t)gridDim.x * KV_WG;
    for (int64_t i = (int64_t)blockIdx.x * KV_WG + threadIdx.x; i < a.n; i += stride) {
        const double ri = a.b[i] - a.v[i];
        r[i] = ri;
        acc[0] += ri * ri;
    }
    block_reduce<double, 1, KV_WG>(acc, red, a.part + (int64_t)blockIdx.x * SSTEP_REC);
}

/* end of a phase: k += s, history (NaN inside the phase), convergence */
__global__ __launch_bounds__(SHARED_WG) void sstep_r_finish(const SStepArgs a, int64_t nparts, int sdim)
{
    __shared__ double red[SHARED_WG];
    __shared__ double tot[1];
    CGState *st = a.st;
    if (st->flag != FLAG_RUN) return;
    sum_records<1, SSTEP_REC>(a.part, nparts, red, tot);
    if (threadIdx.x != 0) return;
    const int k = st->k + sdim;
    const double rho = sqrt(tot[0]);
    for (int j = k - sdim + 1; j < k; ++j) a.hist[j] = __builtin_nan("");
    a.hist[k] = rho;
    st->k = k;
    a.ks->phase += 1;
    if (!isfinite(rho))
        st->flag = FLAG_BREAK;
    else if (rho < st->eps)
        st->flag = FLAG_CONV;
}

template <int S>
static hipError_t sstep_blocks(const SStepArgs &a, hipStream_t s)
{
    const int nb = vec_blocks(a.n);
    hipLaunchKernelGGL(sstep_c_kernel<S>, dim3(nb), dim3(KV_WG), 0, s, a);
    hipLaunchKernelGGL(sstep_b_finish<S>, dim3(1), dim3(SHARED_WG), 0, s, a, (int64_t)nb);
    hipLaunchKernelGGL(sstep_p_kernel<S>, dim3(nb), dim3(KV_WG), 0, s, a);
    hipLaunchKernelGGL(sstep_a_finish<S>, dim3(1), dim3(SHARED_WG), 0, s, a, (int64_t)nb);
    hipLaunchKernelGGL(sstep_x_kernel<S>, dim3(nb), dim3(KV_WG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sstep_blocks(const SStepArgs &a, int sdim, hipStream_t s)
{
    static_assert(SSTEP_MAX * SSTEP_MAX + SSTEP_MAX <= SSTEP_REC, "record too small");
    switch (sdim) {
    case 1: return sstep_blocks<1>(a, s);
    case 2: return sstep_blocks<2>(a, s);
    case 3: return sstep_blocks<3>(a, s);
    case 4: return sstep_blocks<4>(a, s);
    case 5: return sstep_blocks<5>(a, s);
    case 6: return sstep_blocks<6>(a, s);
    case 7: return sstep_blocks<7>(a, s);
    case 8: return sstep_blocks<8>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sstep_residual(const SStepArgs &a, int sdim, hipStream_t s)
{
    if (sdim < 1 || sdim > SSTEP_MAX) return hipErrorInvalidValue;
    const int nb = vec_blocks(a.n);
    hipLaunchKernelGGL(sstep_r_kernel, dim3(nb), dim3(KV_WG), 0, s, a);
    hipLaunchKernelGGL(sstep_r_finish, dim3(1), dim3(SHARED_WG), 0, s, a, (int64_t)nb, sdim);
    return hipGetLastError();
}

}  // namespace mfcg
