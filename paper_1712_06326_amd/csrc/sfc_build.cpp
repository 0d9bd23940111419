// Host orchestration of the SFC multi-index: build (Sections II, II.A-C) and
// query (Fig. 1 b-d). All arithmetic runs in the kernels; the host derives
// the static geometry tables (pixel subsets, element offsets), sizes the
// buffers and plans the sort passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "build.hpp"
#include "index.hpp"
#include "mfma_scan.hpp"
#include "proj.hpp"
#include "query.hpp"

namespace sfc {

bool scan_supported(int nd, int K, int C);
bool rescore_supported(int nd, int K, int C);

namespace {

// Pixel subsets (Fig. 2): anchors at the corners and edge midpoints of the
// patch, a in {0,1,2}^nd without the centre, lexicographic with axis 0
// slowest; each takes every pixel whose squared distance to the anchor is at
// most the ceil(0.6*K^nd)-th smallest one (ties at the cut included).
void make_subsets(int nd, int K, std::vector<int32_t>& npix, std::vector<int32_t>& pix) {
    int Kd = 1;
    for (int i = 0; i < nd; i++) Kd *= K;
    const int h = (K - 1) / 2;
    const int need = (6 * Kd + 9) / 10;
    int n3 = 1;
    for (int i = 0; i < nd; i++) n3 *= 3;
    npix.clear();
    pix.clear();
    std::vector<int> d2(Kd), sorted(Kd);
    for (int a = 0; a < n3; a++) {
        int anchor[kMaxDims];
        bool centre = true;
        for (int i = nd - 1, r = a; i >= 0; i--, r /= 3) {
            anchor[i] = (r % 3) * h;
            if (r % 3 != 1) centre = false;
        }
        if (centre) continue;
        for (int rho = 0; rho < Kd; rho++) {
            int acc = 0;
            for (int i = nd - 1, r = rho; i >= 0; i--, r /= K) {
                const int dd = r % K - anchor[i];
                acc += dd * dd;
            }
            d2[rho] = acc;
        }
        sorted = d2;
        std::nth_element(sorted.begin(), sorted.begin() + (need - 1), sorted.end());
        const int cut = sorted[need - 1];
        int cnt = 0;
        const size_t base = pix.size();
        pix.resize(base + Kd, -1);
        for (int rho = 0; rho < Kd; rho++)
            if (d2[rho] <= cut) pix[base + cnt++] = rho;
        npix.push_back(cnt);
    }
}

template <typename T>
sfc_status upload(T** dst, const std::vector<T>& src, const char* what, hipStream_t st) {
    SFC_TRY(dev_alloc((void**)dst, src.size() * sizeof(T), what));
    SFC_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return SFC_OK;
}

// Stream-ordered temporaries of one build step, freed on the stream at
// scope exit (no wait for other streams).
struct Temp {
    hipStream_t st;
    std::vector<void*> ptrs;
    explicit Temp(hipStream_t s) : st(s) {}
    sfc_status alloc(void** p, size_t bytes, const char* what) {
        SFC_TRY(tmp_alloc(p, bytes, what, st));
        ptrs.push_back(*p);
        return SFC_OK;
    }
    ~Temp() {
        for (void* p : ptrs) tmp_free(p, st);
    }
    Temp(const Temp&) = delete;
    Temp& operator=(const Temp&) = delete;
};

__global__ void wtw_kernel(const int8_t* __restrict__ basis, const int32_t* __restrict__ msz,
                           int S, int mmax, int D, int64_t* __restrict__ wtw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S * D * D) return;
    const int s = i / (D * D), d = (i / D) % D, f = i % D;
    const int8_t* w = basis + (int64_t)s * mmax * D;
    int64_t acc = 0;
    for (int r = 0; r < msz[s]; r++) acc += (int64_t)w[r * D + d] * w[r * D + f];
    wtw[i] = acc;
}

// ws[s][d] = sum over the subset's elements r of w[r][d] * sum[elem r]
__global__ void basis_sums_kernel(const int8_t* __restrict__ basis, const int32_t* __restrict__ msz,
                                  const int32_t* __restrict__ elems,
                                  const uint64_t* __restrict__ sum, int S, int mmax, int D,
                                  int64_t* __restrict__ ws) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S * D) return;
    const int s = i / D, d = i % D;
    const int8_t* w = basis + (int64_t)s * mmax * D;
    int64_t acc = 0;
    for (int r = 0; r < msz[s]; r++) acc += (int64_t)w[r * D + d] * (int64_t)sum[elems[s * mmax + r]];
    ws[i] = acc;
}

__global__ void zero_bytes_kernel(uint8_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

sfc_status zero(void* p, size_t bytes, hipStream_t st) {
    if (bytes == 0) return SFC_OK;
    zero_bytes_kernel<<<(unsigned)((bytes + 255) / 256), 256, 0, st>>>((uint8_t*)p, (int64_t)bytes);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFC_OK : check_hip(e, "zero_bytes_kernel");
}

__global__ void cols_i32_to_i64_kernel(const int32_t* __restrict__ y, int64_t n, int ystride,
                                       int col0, int D, int64_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * D) return;
    const int64_t r = i / D;
    out[i] = y[r * ystride + col0 + (i - r * D)];
}

__global__ void export_kernel(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ ids,
                              int64_t n, int W64, uint64_t* __restrict__ kout,
                              int64_t* __restrict__ iout) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int w = 0; w < W64; w++) kout[i * W64 + w] = keys[(int64_t)w * n + i];
    iout[i] = ids[i];
}

QueryIndexView view_of(const sfc_index* ix) {
    QueryIndexView v{};
    const Grid& g = ix->g;
    v.nd = g.nd;
    v.K = g.K;
    v.C = g.C;
    v.Kd = g.Kd;
    v.rows = g.rows;
    v.h = g.h;
    for (int i = 0; i < kMaxDims; i++) {
        v.shape[i] = g.shape[i];
        v.stride[i] = g.stride[i];
    }
    v.S = ix->S;
    v.D = ix->D;
    v.L = ix->L;
    v.b = ix->b;
    v.curve = ix->opt.curve;
    v.W64 = ix->W64;
    v.window = ix->opt.window;
    v.mmax = ix->mmax;
    v.R = ix->R;
    v.n = ix->n;
    v.nsub = ix->nsub;
    v.qparams = ix->qparams;
    v.npix = ix->npix;
    v.pix = ix->pix;
    v.basis = ix->basis;
    v.wtw = ix->wtw;
    v.ws = ix->ws;
    v.smask = ix->smask;
    v.sum = reinterpret_cast<const uint64_t*>(ix->sum);
    v.lo = ix->lo;
    v.span = ix->span;
    v.keys = ix->keys;
    v.ids = ix->ids;
    return v;
}

}  // namespace

// Sorts narr consecutive arrays of n (key, id) pairs (keys [narr][W64][n],
// ids [narr][n]) by (key, position), stable. The arrays are sorted in groups
// whose ping-pong copies fit a fixed budget, each group with the union of
// its arrays' varying 8-bit digit positions below nbits.
sfc_status sort_key_arrays(uint64_t* keys, uint32_t* ids, int64_t n, int W64, int narr,
                           int nbits, hipStream_t st) {
    if (n <= 1 || narr <= 0) return SFC_OK;
    Temp tmp(st);
    uint64_t* varying = nullptr;
    SFC_TRY(tmp.alloc((void**)&varying, (size_t)narr * W64 * 8, "varying bits"));
    SFC_TRY(zero(varying, (size_t)narr * W64 * 8, st));
    SFC_TRY(launch_varying_bits(keys, n, W64, narr, varying, st));
    std::vector<uint64_t> hv((size_t)narr * W64);
    SFC_HIP(hipMemcpyAsync(hv.data(), varying, hv.size() * 8, hipMemcpyDeviceToHost, st));
    SFC_HIP(hipStreamSynchronize(st));
    const size_t per_arr = sort_scratch_bytes(n, W64, 1);
    int group = (int)std::max<size_t>(1, std::min<size_t>(narr, (size_t(8) << 30) / per_arr));
    void* sscratch = nullptr;
    SFC_TRY(tmp.alloc(&sscratch, sort_scratch_bytes(n, W64, group), "sort scratch"));
    for (int a0 = 0; a0 < narr; a0 += group) {
        const int na = std::min(group, narr - a0);
        SortPlan plan{};
        for (int pb = 0; pb < nbits; pb += 8) {
            const int w = W64 - 1 - (pb >> 6);
            uint64_t bits = 0;
            for (int a = a0; a < a0 + na; a++) bits |= (hv[(size_t)a * W64 + w] >> (pb & 63)) & 0xffull;
            if (bits) plan.pass_bits[plan.n_passes++] = pb;
        }
        SFC_TRY(radix_sort(keys + (size_t)a0 * W64 * n, ids + (size_t)a0 * n, n, W64, na, plan,
                           sscratch, st));
    }
    // the scratch is freed on return
    SFC_HIP(hipStreamSynchronize(st));
    return SFC_OK;
}

sfc_status check_sfc_args(const sfc_geometry* g, int K, int D, int L, const sfc_options& o) {
    if (D < 1) return fail(SFC_EINVAL, "reduced_dim must be >= 1");
    if (L < 1) return fail(SFC_EINVAL, "n_curves must be >= 1");
    if (L > D + 1) return fail(SFC_EINVAL, "n_curves must be <= reduced_dim + 1 (shift headroom)");
    if ((int64_t)D * o.key_bits > 256) return fail(SFC_EINVAL, "reduced_dim * key_bits above 256");
    if (D > 12 && D != 16) return fail(SFC_EUNSUPPORTED, "reduced_dim must be 1..12 or 16");
    if ((int64_t)L * o.window > 2048) return fail(SFC_EUNSUPPORTED, "n_curves * window above 2048");
    if (!scan_supported(g->ndim, K, g->channels) || !rescore_supported(g->ndim, K, g->channels))
        return fail(SFC_EUNSUPPORTED, "no kernels for this (ndim, K, channels)");
    int Kd = 1;
    for (int i = 0; i < g->ndim; i++) Kd *= K;
    if (D > (6 * Kd + 9) / 10 * g->channels)
        return fail(SFC_EINVAL, "reduced_dim larger than a subset's element count");
    return SFC_OK;
}

// Byte codes of the volume and their parameters (shared by the index build
// and the reduced-precision scan), computed once per handle.
sfc_status ensure_quantized(sfc_index* ix, const uint8_t* mask) {
    if (ix->xq) return SFC_OK;
    const Grid& g = ix->g;
    SFC_TRY(dev_alloc((void**)&ix->xq, (size_t)g.nvox * g.C, "quantised volume"));
    SFC_TRY(dev_alloc((void**)&ix->qparams, 4 * sizeof(float), "quantisation parameters"));
    float qp[2];
    {
        TmpBuf mm(ix->st);
        SFC_TRY(mm.alloc(2 * kQuantBlocks * sizeof(uint32_t), "min/max"));
        SFC_TRY(launch_quantize(ix->vol, mask, g, ix->xq, ix->qparams,
                                static_cast<uint32_t*>(mm.ptr), ix->st));
        SFC_HIP(hipMemcpyAsync(qp, ix->qparams, sizeof(qp), hipMemcpyDeviceToHost, ix->st));
        SFC_HIP(hipStreamSynchronize(ix->st));
    }
    ix->vmin = qp[0];
    ix->qscale = qp[1];
    return SFC_OK;
}

sfc_status code_checksum(sfc_index* ix, uint64_t* out_host) {
    SFC_TRY(ensure_quantized(ix, ix->mask_copy));
    uint64_t* d = nullptr;
    SFC_TRY(dev_alloc((void**)&d, sizeof(uint64_t), "checksum"));
    sfc_status s = launch_code_checksum(ix->xq, ix->mask_copy, ix->g.nvox, ix->g.C, d, ix->st);
    if (s == SFC_OK) {
        hipError_t e = hipMemcpyAsync(out_host, d, sizeof(uint64_t), hipMemcpyDeviceToHost, ix->st);
        if (e == hipSuccess) e = hipStreamSynchronize(ix->st);
        if (e != hipSuccess) s = check_hip(e, "checksum");
    }
    dev_free(d);
    return s;
}

sfc_status ensure_elem_offsets(sfc_index* ix) {
    if (ix->elem_off) return SFC_OK;
    const Grid& g = ix->g;
    const int P = g.Kd * g.C;
    const int Pp = (P + 15) / 16 * 16;
    std::vector<int32_t> eoff(Pp, 0);
    for (int e = 0; e < P; e++) {
        int rho = e / g.C;
        int64_t off = 0;
        for (int i = g.nd - 1; i >= 0; i--, rho /= g.K) off += (int64_t)(rho % g.K - g.h) * g.stride[i];
        eoff[e] = (int32_t)(off * g.C + e % g.C);
    }
    return upload(&ix->elem_off, eoff, "element offsets", ix->st);
}

void release_sfc(sfc_index* ix) {
    void* ps[] = {ix->xq, ix->sum, ix->npix, ix->pix, ix->basis, ix->lo, ix->span, ix->keys,
                  ix->ids, ix->proj_w, ix->wtw, ix->ws, ix->smask, ix->qparams, ix->elems,
                  ix->msz, ix->elem_off, ix->mfma_B, ix->mask_copy};
    for (void* p : ps) dev_free(p);
    ix->xq = nullptr;
    ix->keys = nullptr;
    ix->ids = nullptr;
}

// W^T W of every basis (the query's least-squares imputation) and the int8
// projection weights with their column sums, from the bases on the device.
sfc_status basis_products(sfc_index* ix, hipStream_t st) {
    const int S = ix->S, D = ix->D, mmax = ix->mmax, P = ix->g.Kd * ix->g.C;
    SFC_TRY(dev_alloc((void**)&ix->wtw, (size_t)S * D * D * 8, "basis gram"));
    wtw_kernel<<<(S * D * D + 255) / 256, 256, 0, st>>>(ix->basis, ix->msz, S, mmax, D, ix->wtw);
    SFC_HIP(hipGetLastError());
    SFC_TRY(dev_alloc((void**)&ix->ws, (size_t)S * D * 8, "basis sums"));
    basis_sums_kernel<<<(S * D + 255) / 256, 256, 0, st>>>(
        ix->basis, ix->msz, ix->elems, reinterpret_cast<const uint64_t*>(ix->sum), S, mmax, D, ix->ws);
    SFC_HIP(hipGetLastError());

    // projection weights (int8) and their column sums
    const int ncols = S * D;
    const int nt = proj_tiles(ncols);
    if (nt > 16) return fail(SFC_EUNSUPPORTED, "subsets * reduced_dim above 512");
    const size_t wbytes = proj_weight_bytes(ncols, P);
    SFC_TRY(dev_alloc(&ix->proj_w, wbytes, "projection weights"));
    SFC_TRY(zero(ix->proj_w, wbytes, st));
    int8_t* W = static_cast<int8_t*>(ix->proj_w);
    SFC_TRY(launch_weights(ix->basis, ix->elems, ix->msz, S, mmax, D, P, ncols, W,
                           reinterpret_cast<int32_t*>(W + (size_t)nt * 32 * proj_depth(P)), st));
    return SFC_OK;
}

// The patch layout and weights of the projection kernel.
void set_proj_weights(const sfc_index* ix, ProjArgs& pa) {
    const int P = ix->g.Kd * ix->g.C;
    pa.P = P;
    pa.Pk = proj_depth(P);
    pa.C = ix->g.C;
    pa.run = ix->g.K * ix->g.C;
    const int8_t* W = static_cast<const int8_t*>(ix->proj_w);
    pa.Wt = W;
    pa.wsum = reinterpret_cast<const int32_t*>(W + (size_t)proj_tiles(ix->S * ix->D) * 32 * pa.Pk);
}

// Host copies of the small parameters; marks the handle as an SFC index.
sfc_status finish_sfc(sfc_index* ix, hipStream_t st) {
    const int S = ix->S, D = ix->D, mmax = ix->mmax;
    ix->h_basis.assign((size_t)S * mmax * D, 0);
    ix->h_lo.assign((size_t)S * D, 0);
    ix->h_span.assign(S, 0);
    float qp[2];
    SFC_HIP(hipMemcpyAsync(ix->h_basis.data(), ix->basis, ix->h_basis.size(), hipMemcpyDeviceToHost, st));
    SFC_HIP(hipMemcpyAsync(ix->h_lo.data(), ix->lo, ix->h_lo.size() * 8, hipMemcpyDeviceToHost, st));
    SFC_HIP(hipMemcpyAsync(ix->h_span.data(), ix->span, ix->h_span.size() * 8, hipMemcpyDeviceToHost, st));
    SFC_HIP(hipMemcpyAsync(qp, ix->qparams, sizeof(qp), hipMemcpyDeviceToHost, st));
    SFC_HIP(hipStreamSynchronize(st));
    ix->vmin = qp[0];
    ix->qscale = qp[1];
    ix->has_sfc = true;
    return SFC_OK;
}

sfc_status curves_from_basis(sfc_index* ix, hipStream_t st);

sfc_status build_sfc(sfc_index* ix, const uint8_t* mask, int D, int L, const int8_t* bases_host,
                     const SavedIndex* saved) {
    const Grid& g = ix->g;
    hipStream_t st = ix->st;
    const int C = g.C, P = g.Kd * C;
    ix->D = D;
    ix->L = L;
    ix->b = ix->opt.key_bits;
    ix->W64 = (D * ix->b + 63) / 64;
    ix->R = (L > 1) ? (int64_t(1) << (ix->b - 1)) : (int64_t(1) << ix->b);

    // static tables: subsets, their elements, element offsets
    make_subsets(g.nd, g.K, ix->h_npix, ix->h_pix);
    ix->S = (int)ix->h_npix.size();
    const int S = ix->S;
    int mmax = 0;
    for (int s = 0; s < S; s++) mmax = std::max(mmax, ix->h_npix[s] * C);
    if (mmax > kMaxSubsetElems)
        return fail(SFC_EUNSUPPORTED, "a subset has more than 518 elements (eigensolver bound)");
    ix->mmax = mmax;
    std::vector<int32_t> elems((size_t)S * mmax, 0), msz(S);
    for (int s = 0; s < S; s++) {
        msz[s] = ix->h_npix[s] * C;
        for (int i = 0; i < ix->h_npix[s]; i++)
            for (int ch = 0; ch < C; ch++) elems[(size_t)s * mmax + i * C + ch] = ix->h_pix[(size_t)s * g.Kd + i] * C + ch;
    }
    const int Pp = (P + 15) / 16 * 16;
    ix->Pp = Pp;
    std::vector<int32_t> eoff(Pp, 0);
    for (int e = 0; e < P; e++) {
        int rho = e / C;
        int64_t off = 0;
        for (int i = g.nd - 1; i >= 0; i--, rho /= g.K) off += (int64_t)(rho % g.K - g.h) * g.stride[i];
        eoff[e] = (int32_t)(off * C + e % C);
    }
    const int KW = (g.Kd + 63) / 64;
    std::vector<uint64_t> smask((size_t)S * KW, 0);
    for (int s = 0; s < S; s++)
        for (int i = 0; i < ix->h_npix[s]; i++) {
            const int rho = ix->h_pix[(size_t)s * g.Kd + i];
            smask[(size_t)s * KW + rho / 64] |= 1ull << (rho % 64);
        }
    SFC_TRY(upload(&ix->smask, smask, "subset pixel masks", st));
    SFC_TRY(upload(&ix->npix, ix->h_npix, "subset sizes", st));
    SFC_TRY(upload(&ix->pix, ix->h_pix, "subset pixels", st));
    SFC_TRY(upload(&ix->elems, elems, "subset elements", st));
    SFC_TRY(upload(&ix->msz, msz, "subset element counts", st));
    if (!ix->elem_off) SFC_TRY(upload(&ix->elem_off, eoff, "element offsets", st));

    // byte quantisation
    SFC_TRY(ensure_quantized(ix, mask));
    if (saved) {
        // a saved index: its statistics and bases, after checking that the
        // rebuilt quantisation and subsample are the ones they came from
        const int64_t stride = std::max<int64_t>(1, (ix->n + (1 << 20) - 1) >> 20);
        const int64_t nsub = (ix->n + stride - 1) / stride;
        if (saved->nsub != nsub || ix->vmin != saved->vmin || ix->qscale != saved->qscale)
            return fail(SFC_EINVAL, "index file was made from another volume or mask");
        if (saved->sum.size() != (size_t)P || saved->basis.size() != (size_t)S * mmax * D ||
            saved->lo.size() != (size_t)S * D || saved->span.size() != (size_t)S)
            return fail(SFC_EINVAL, "index file: array sizes do not match its header");
        ix->nsub = nsub;
        SFC_TRY(upload(reinterpret_cast<uint64_t**>(&ix->sum), saved->sum, "sample sums", st));
        SFC_TRY(upload(&ix->basis, saved->basis, "bases", st));
        SFC_TRY(curves_from_basis(ix, st));
        if (ix->h_lo != saved->lo || ix->h_span != saved->span)
            return fail(SFC_EINVAL, "index file: its grid does not match the rebuilt projections");
        return SFC_OK;
    }
    {
        // the statistics and the eigensolver's matrices are freed before
        // the curves are built
        Temp tmp(st);

        // integer statistics over the strided subsample
        const int64_t stride = (ix->n + (1 << 20) - 1) >> 20;
        const int64_t st1 = stride < 1 ? 1 : stride;
        ix->nsub = (ix->n + st1 - 1) / st1;
        const int64_t nsp4 = (ix->nsub + 3) / 4;
        uint32_t* Xt = nullptr;
        uint64_t* gram = nullptr;
        SFC_TRY(tmp.alloc((void**)&Xt, (size_t)P * nsp4 * 4, "sample matrix"));
        SFC_TRY(dev_alloc((void**)&ix->sum, (size_t)P * 8, "sample sums"));
        SFC_TRY(zero(ix->sum, (size_t)P * 8, st));
        SFC_TRY(tmp.alloc((void**)&gram, (size_t)P * P * 8, "gram matrix"));
        SFC_TRY(zero(gram, (size_t)P * P * 8, st));
        SFC_TRY(launch_gather_samples(ix->xq, ix->dict, st1, ix->nsub, ix->elem_off, P, C, Xt, nsp4, st));
        SFC_TRY(launch_gram(Xt, P, nsp4, reinterpret_cast<uint64_t*>(ix->sum), gram, st));

        // basis per subset
        SFC_TRY(dev_alloc((void**)&ix->basis, (size_t)S * mmax * D, "bases"));
        if (!bases_host) {
            double *A = nullptr, *V = nullptr;
            void* B = nullptr;
            int32_t* sweeps = nullptr;
            const size_t mat = (size_t)S * mmax * mmax * sizeof(double);
            SFC_TRY(tmp.alloc((void**)&A, mat, "covariance matrices"));
            SFC_TRY(tmp.alloc((void**)&V, mat, "eigenvectors"));
            SFC_TRY(tmp.alloc(&B, jacobi_scratch_bytes(S, mmax), "eigensolver scratch"));
            SFC_TRY(tmp.alloc((void**)&sweeps, S * sizeof(int32_t), "sweep counts"));
            SFC_TRY(launch_cov_matrix(reinterpret_cast<uint64_t*>(ix->sum), gram, ix->nsub, P,
                                      ix->elems, ix->msz, S, mmax, A, st));
            SFC_TRY(launch_jacobi(A, V, B, ix->msz, S, mmax, sweeps, st));
            SFC_TRY(launch_basis(A, V, ix->msz, S, mmax, D, ix->basis, st));
        } else {
            std::vector<int8_t> hb((size_t)S * mmax * D, 0);
            size_t off = 0;
            for (int s = 0; s < S; s++) {
                std::memcpy(&hb[(size_t)s * mmax * D], bases_host + off, (size_t)msz[s] * D);
                off += (size_t)msz[s] * D;
            }
            SFC_HIP(hipMemcpyAsync(ix->basis, hb.data(), hb.size(), hipMemcpyHostToDevice, st));
            SFC_HIP(hipStreamSynchronize(st));
        }
        SFC_HIP(hipStreamSynchronize(st));
    }
    return curves_from_basis(ix, st);
}

// Everything that follows from the bases: projection weights, principal
// coordinates of every dictionary patch, grid origin and span, keys of
// every (subset, curve), the sort.
sfc_status curves_from_basis(sfc_index* ix, hipStream_t st) {
    const int S = ix->S, D = ix->D, L = ix->L;
    Temp tmp(st);
    SFC_TRY(basis_products(ix, st));
    const int ncols = S * D;
    int32_t *cmin = nullptr, *cmax = nullptr;
    SFC_TRY(tmp.alloc((void**)&cmin, ncols * 4, "column minima"));
    SFC_TRY(tmp.alloc((void**)&cmax, ncols * 4, "column maxima"));
    SFC_TRY(launch_init_minmax(cmin, cmax, ncols, st));
    const int64_t chunk = std::min<int64_t>(ix->n, int64_t(1) << 24);
    int32_t* y = nullptr;
    SFC_TRY(tmp.alloc((void**)&y, (size_t)chunk * ncols * 4, "principal coordinates"));
    ProjArgs pa{};
    pa.xq = ix->xq;
    pa.dict = ix->dict;
    pa.elem_off = ix->elem_off;
    set_proj_weights(ix, pa);
    pa.ncols = ncols;
    pa.ystride = ncols;
    pa.colmin = cmin;
    pa.colmax = cmax;
    const bool one_chunk = chunk == ix->n;
    for (int64_t r0 = 0; r0 < ix->n; r0 += chunk) {
        pa.r0 = r0;
        pa.cnt = std::min(chunk, ix->n - r0);
        pa.y = one_chunk ? y : nullptr;
        SFC_TRY(launch_projection(pa, st));
    }
    SFC_TRY(dev_alloc((void**)&ix->lo, (size_t)S * D * 8, "grid origin"));
    SFC_TRY(dev_alloc((void**)&ix->span, (size_t)S * 8, "grid span"));
    SFC_TRY(launch_span(cmin, cmax, S, D, ix->lo, ix->span, st));

    // keys of every (subset, curve)
    const size_t nkeys = (size_t)S * L * ix->W64 * ix->n;
    SFC_TRY(dev_alloc((void**)&ix->keys, nkeys * 8, "curve keys"));
    SFC_TRY(dev_alloc((void**)&ix->ids, (size_t)S * L * ix->n * 4, "curve ids"));
    KeyArgs ka{};
    ka.y = y;
    ka.ystride = ncols;
    ka.n = ix->n;
    ka.dict = ix->dict;
    ka.S = S;
    ka.D = D;
    ka.L = L;
    ka.b = ix->b;
    ka.curve = ix->opt.curve;
    ka.W64 = ix->W64;
    ka.R = ix->R;
    ka.lo = ix->lo;
    ka.span = ix->span;
    ka.keys = ix->keys;
    ka.ids = ix->ids;
    for (int64_t r0 = 0; r0 < ix->n; r0 += chunk) {
        pa.r0 = r0;
        pa.cnt = std::min(chunk, ix->n - r0);
        if (!one_chunk) {
            pa.y = y;
            pa.colmin = nullptr;
            pa.colmax = nullptr;
            SFC_TRY(launch_projection(pa, st));
        }
        ka.r0 = r0;
        ka.cnt = pa.cnt;
        SFC_TRY(launch_keys(ka, st));
    }

    // sort every (subset, curve) by (key, id)
    SFC_TRY(sort_key_arrays(ix->keys, ix->ids, ix->n, ix->W64, S * L, D * ix->b, st));

    return finish_sfc(ix, st);
}

namespace {
// Layout of the index query's temporaries: row masks, coordinates, keys,
// window starts, subsets, packed minima and tickets of the split rescoring
// (each at a 256-byte boundary).
struct IndexQueryLayout {
    size_t rm, co, k, w, s, pb, tk, total;
    IndexQueryLayout(const sfc_index* ix, int64_t Q) {
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t at = off;
            off += (bytes + 255) & ~size_t(255);
            return at;
        };
        rm = take((size_t)scan_qpad(Q) * ix->g.rows * sizeof(uint32_t));
        co = take((size_t)Q * 8 * ix->D);
        k = take((size_t)Q * 8 * ix->L * ix->W64);
        w = take((size_t)Q * 8 * ix->L);
        s = take((size_t)Q * 4);
        pb = take((size_t)Q * 8);
        tk = take((size_t)Q * 4);
        total = off;
    }
};
}  // namespace

size_t index_query_bytes(const sfc_index* ix, int64_t Q) { return IndexQueryLayout(ix, Q).total; }

sfc_status query_index(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q, int64_t* best_id,
                       float* best_cost, int64_t* cand, int32_t* ncand) {
    // the handle's grow-only buffer: allocated on first use, reused after
    SFC_TRY(ix->qtmp.reserve(index_query_bytes(ix, Q), "query scratch"));
    return query_index_on(ix, t, m, Q, ix->qtmp.ptr, best_id, best_cost, cand, ncand);
}

sfc_status query_index_on(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q, void* buf,
                          int64_t* best_id, float* best_cost, int64_t* cand, int32_t* ncand,
                          const LoopApply* apply) {
    hipStream_t st = ix->st;
    const int64_t qpad = scan_qpad(Q);
    const IndexQueryLayout lay(ix, Q);
    char* base = static_cast<char*>(buf);
    uint32_t* rm = reinterpret_cast<uint32_t*>(base + lay.rm);
    double* coords = reinterpret_cast<double*>(base + lay.co);
    uint64_t* qkeys = reinterpret_cast<uint64_t*>(base + lay.k);
    int64_t* wstart = reinterpret_cast<int64_t*>(base + lay.w);
    int32_t* qsub = reinterpret_cast<int32_t*>(base + lay.s);
    uint64_t* qbest = reinterpret_cast<uint64_t*>(base + lay.pb);
    int32_t* qticket = reinterpret_cast<int32_t*>(base + lay.tk);
    const QueryIndexView v = view_of(ix);
    SFC_TRY(ix->timer.begin("prologue_kernel", st));
    SFC_TRY(launch_query_prologue(v, t, m, Q, qsub, coords, qkeys, rm, qpad, qbest, qticket, st));
    SFC_TRY(ix->timer.end(st));
    SFC_TRY(ix->timer.begin("search_kernel", st));
    SFC_TRY(launch_query_search(v, qsub, qkeys, Q, wstart, st));
    SFC_TRY(ix->timer.end(st));
    SFC_TRY(ix->timer.begin("rescore_kernel", st));
    SFC_TRY(launch_query_rescore(v, ix->vol, t, rm, qpad, qsub, wstart, Q, best_id, best_cost, cand,
                                 ncand, ix->opt.norm, qbest, qticket, apply, st));
    return ix->timer.end(st);
}

sfc_status query_knn(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q, int k, int mu,
                     int64_t* best_id, float* best_cost, int64_t* cand, int32_t* ncand) {
    const Grid& g = ix->g;
    hipStream_t st = ix->st;
    const int64_t qpad = scan_qpad(Q);
    const size_t need = (size_t)qpad * g.rows * 4 + 64 +
                        (size_t)Q * (4 + 8 * ix->D + 8 * ix->L * ix->W64 + 4 * k + 4 + 4 + 1) + 1024;
    SFC_TRY(ix->qtmp.reserve(need, "k-NN query scratch"));
    char* p = static_cast<char*>(ix->qtmp.ptr);
    auto take = [&](size_t bytes) {
        char* r = p;
        p += (bytes + 63) & ~size_t(63);
        return r;
    };
    uint32_t* rm = reinterpret_cast<uint32_t*>(take((size_t)qpad * g.rows * 4));
    double* coords = reinterpret_cast<double*>(take((size_t)Q * 8 * ix->D));
    uint64_t* qkeys = reinterpret_cast<uint64_t*>(take((size_t)Q * 8 * ix->L * ix->W64));
    int32_t* qsub = reinterpret_cast<int32_t*>(take((size_t)Q * 4));
    uint32_t* list = reinterpret_cast<uint32_t*>(take((size_t)Q * 4 * k));
    int32_t* cnt = reinterpret_cast<int32_t*>(take((size_t)Q * 4));
    int32_t* thr = reinterpret_cast<int32_t*>(take((size_t)Q * 4));
    uint8_t* fb = reinterpret_cast<uint8_t*>(take((size_t)Q));
    uint64_t* flag = reinterpret_cast<uint64_t*>(take(8));
    SFC_TRY(launch_fill_u64(flag, 1, 0ull, st));
    const QueryIndexView v = view_of(ix);
    SFC_TRY(ix->timer.begin("prologue_kernel", st));
    SFC_TRY(launch_query_prologue(v, t, m, Q, qsub, coords, qkeys, rm, qpad, nullptr, nullptr, st));
    SFC_TRY(ix->timer.end(st));
    SFC_TRY(ix->timer.begin("knn_kernel", st));
    SFC_TRY(launch_knn(v, qsub, coords, Q, k, mu, list, cnt, thr,
                       reinterpret_cast<unsigned int*>(flag), st));
    SFC_TRY(ix->timer.end(st));
    SFC_TRY(ix->timer.begin("list_rescore_kernel", st));
    SFC_TRY(launch_list_rescore(g, ix->vol, t, rm, qpad, list, cnt, thr, k, Q, best_id, best_cost,
                                fb, ix->opt.norm, st));
    SFC_TRY(ix->timer.end(st));
    SFC_TRY(launch_knn_cand(list, cnt, Q, k, cand, ncand, st));
    uint64_t over = 0;
    SFC_HIP(hipMemcpyAsync(&over, flag, 8, hipMemcpyDeviceToHost, st));
    SFC_HIP(hipStreamSynchronize(st));
    if (over) return fail(SFC_EDEVICE, "k-NN query: a traversal stack overflowed");
    return SFC_OK;
}

sfc_status query_coords(sfc_index* ix, const float* t, const uint8_t* m, int64_t Q, int32_t* subset,
                        double* coords) {
    const size_t need = (size_t)Q * 8 * ix->L * ix->W64 + 256;
    SFC_TRY(ix->qtmp.reserve(need, "query scratch"));
    uint64_t* qkeys = static_cast<uint64_t*>(ix->qtmp.ptr);
    const QueryIndexView v = view_of(ix);
    return launch_query_prologue(v, t, m, Q, subset, coords, qkeys, nullptr, 0, nullptr, nullptr,
                                 ix->st);
}

}  // namespace sfc

using namespace sfc;

extern "C" {

sfc_status sfc_index_quantized(const sfc_index* ix, uint8_t* xq) {
    clear_error();
    if (!ix || !xq) return fail(SFC_EINVAL, "null pointer");
    if (!ix->has_sfc) return fail(SFC_EINVAL, "no SFC index on this handle");
    SFC_HIP(hipMemcpyAsync(xq, ix->xq, (size_t)ix->g.nvox * ix->g.C, hipMemcpyDeviceToDevice, ix->st));
    return SFC_OK;
}

sfc_status sfc_index_get_basis(const sfc_index* ix, int32_t subset, int8_t* out, int32_t* rows) {
    clear_error();
    if (!ix || !out || !rows) return fail(SFC_EINVAL, "null pointer");
    if (!ix->has_sfc) return fail(SFC_EINVAL, "no SFC index on this handle");
    if (subset < 0 || subset >= ix->S) return fail(SFC_EINVAL, "subset out of range");
    const int m = ix->h_npix[subset] * ix->g.C;
    std::memcpy(out, &ix->h_basis[(size_t)subset * ix->mmax * ix->D], (size_t)m * ix->D);
    *rows = m;
    return SFC_OK;
}

sfc_status sfc_index_get_params(const sfc_index* ix, int32_t subset, int64_t* lo, int64_t* span) {
    clear_error();
    if (!ix || !lo || !span) return fail(SFC_EINVAL, "null pointer");
    if (!ix->has_sfc) return fail(SFC_EINVAL, "no SFC index on this handle");
    if (subset < 0 || subset >= ix->S) return fail(SFC_EINVAL, "subset out of range");
    std::memcpy(lo, &ix->h_lo[(size_t)subset * ix->D], (size_t)ix->D * 8);
    *span = ix->h_span[subset];
    return SFC_OK;
}

sfc_status sfc_index_projection(const sfc_index* ix, int32_t subset, int64_t* y) {
    clear_error();
    if (!ix || !y) return fail(SFC_EINVAL, "null pointer");
    if (!ix->has_sfc) return fail(SFC_EINVAL, "no SFC index on this handle");
    if (subset < 0 || subset >= ix->S) return fail(SFC_EINVAL, "subset out of range");
    const int ncols = ix->S * ix->D;
    const int64_t chunk = std::min<int64_t>(ix->n, int64_t(1) << 22);
    int32_t* buf = nullptr;
    SFC_TRY(dev_alloc((void**)&buf, (size_t)chunk * ncols * 4, "projection export"));
    ProjArgs pa{};
    pa.xq = ix->xq;
    pa.dict = ix->dict;
    pa.elem_off = ix->elem_off;
    set_proj_weights(ix, pa);
    pa.ncols = ncols;
    pa.ystride = ncols;
    pa.y = buf;
    sfc_status s = SFC_OK;
    for (int64_t r0 = 0; r0 < ix->n && s == SFC_OK; r0 += chunk) {
        pa.r0 = r0;
        pa.cnt = std::min(chunk, ix->n - r0);
        s = launch_projection(pa, ix->st);
        if (s == SFC_OK) {
            cols_i32_to_i64_kernel<<<(unsigned)((pa.cnt * ix->D + 255) / 256), 256, 0, ix->st>>>(
                buf, pa.cnt, ncols, subset * ix->D, ix->D, y + r0 * ix->D);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) s = check_hip(e, "cols_i32_to_i64_kernel");
        }
    }
    hipError_t e = hipStreamSynchronize(ix->st);
    dev_free(buf);
    if (s == SFC_OK && e != hipSuccess) s = check_hip(e, "projection export");
    return s;
}

sfc_status sfc_index_export(const sfc_index* ix, int32_t subset, int32_t curve, uint64_t* keys,
                            int64_t* ids) {
    clear_error();
    if (!ix || !keys || !ids) return fail(SFC_EINVAL, "null pointer");
    if (!ix->has_sfc) return fail(SFC_EINVAL, "no SFC index on this handle");
    if (subset < 0 || subset >= ix->S || curve < 0 || curve >= ix->L)
        return fail(SFC_EINVAL, "subset or curve out of range");
    const int64_t a = (int64_t)subset * ix->L + curve;
    export_kernel<<<(unsigned)((ix->n + 255) / 256), 256, 0, ix->st>>>(
        ix->keys + a * ix->W64 * ix->n, ix->ids + a * ix->n, ix->n, ix->W64, keys, ids);
    SFC_HIP(hipGetLastError());
    return SFC_OK;
}

}  // extern "C"
