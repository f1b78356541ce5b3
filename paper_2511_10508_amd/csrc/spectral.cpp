// Semi-implicit Fourier spectral step of libpfmi (PF_SPECTRAL, Models A and
// B): the paper separates the linear terms, solved in Fourier space, from the
// nonlinear ones, evolved in real space (Sec. "Construction of Semi-Implicit
// Fourier Spectral Scheme").  One step of the state buf[par]:
//   1. g = explicit term of buf[par], written into buf[par ^ 1] (free until
//      step 4 overwrites it);
//   2. real-to-complex transforms g -> nh and, only when the kept spectrum
//      is not that of buf[par] (first step, or the state was set from
//      outside), buf[par] -> uh;
//   3. implicit update (k_spec_update): the next state's spectrum / N, kept
//      in uh and also written over nh;
//   4. complex-to-real transform nh -> buf[par ^ 1] (it may overwrite nh).
// So a run of steps takes two transforms per step, not three.  The
// transforms are hipFFT plans on the library's pitched field layout (rows of
// `pitch` elements), so no repacking pass is needed.
#include <hipfft/hipfft.h>

#include <cmath>

#include "pf_runtime.h"

namespace pf {

struct Spectral {
    hipfftHandle fwd = 0, inv = 0;
    bool have_fwd = false, have_inv = false;
    void *uh = nullptr, *nh = nullptr;  // half spectra, nxh * ny * nz complex values
    SpecArgs args{};
    int kept_par = -1;  // buffer whose state's spectrum / N is in uh (-1: none)
};

void spectral_invalidate(Model *m)
{
    if (m && m->spec) static_cast<Spectral *>(m->spec)->kept_par = -1;
}

static pf_status fft_fail(hipfftResult r, const char *what)
{
    return fail(PF_ERR_DEVICE, std::string(what) + " failed (hipFFT status " +
                                   std::to_string((int)r) + ")");
}

void spectral_release(Model *m)
{
    Spectral *sp = static_cast<Spectral *>(m->spec);
    if (!sp) return;
    if (sp->have_fwd) (void)hipfftDestroy(sp->fwd);
    if (sp->have_inv) (void)hipfftDestroy(sp->inv);
    if (sp->uh) (void)hipFree(sp->uh);
    if (sp->nh) (void)hipFree(sp->nh);
    delete sp;
    m->spec = nullptr;
}

// Bytes of the two half spectra of a descriptor.
uint64_t spectral_bytes(const pf_desc *d)
{
    const uint64_t cb = d->precision == PF_FP32 ? 8 : 16;
    return 2ull * (uint64_t)(d->n[0] / 2 + 1) * (uint64_t)d->n[1] * (uint64_t)d->n[2] * cb;
}

pf_status spectral_setup(Model *m)
{
    if (m->spec) return PF_OK;
    const pf_desc &d = m->desc;
    Spectral *sp = new Spectral();
    m->spec = sp;
    const int64_t nx = d.n[0], ny = d.n[1], nz = d.n[2], nxh = nx / 2 + 1;
    const size_t cbytes = (size_t)nxh * ny * nz * (m->fp32 ? 8 : 16);
    hipError_t e = hipMalloc(&sp->uh, cbytes);
    if (e == hipSuccess) e = hipMalloc(&sp->nh, cbytes);
    if (e != hipSuccess) {
        spectral_release(m);
        hip_fail(e, "hipMalloc(spectra)");
        return PF_ERR_NOMEM;
    }
    // transform sizes, slowest axis first; the real side has rows of `pitch`
    const int rank = d.ndim;
    int n[3], rin[3], cin[3];
    const int64_t ext[3] = {nz, ny, nx};
    for (int i = 0; i < rank; ++i) {
        n[i] = (int)ext[3 - rank + i];
        rin[i] = n[i];
        cin[i] = n[i];
    }
    rin[rank - 1] = (int)m->pitch;
    cin[rank - 1] = (int)nxh;
    const int rdist = (int)m->elems, cdist = (int)(nxh * ny * nz);
    const hipfftType tf = m->fp32 ? HIPFFT_R2C : HIPFFT_D2Z;
    const hipfftType ti = m->fp32 ? HIPFFT_C2R : HIPFFT_Z2D;
    hipfftResult r = hipfftPlanMany(&sp->fwd, rank, n, rin, 1, rdist, cin, 1, cdist, tf, 1);
    if (r != HIPFFT_SUCCESS) {
        spectral_release(m);
        return fft_fail(r, "hipfftPlanMany(forward)");
    }
    sp->have_fwd = true;
    r = hipfftPlanMany(&sp->inv, rank, n, cin, 1, cdist, rin, 1, rdist, ti, 1);
    if (r != HIPFFT_SUCCESS) {
        spectral_release(m);
        return fft_fail(r, "hipfftPlanMany(inverse)");
    }
    sp->have_inv = true;
    r = hipfftSetStream(sp->fwd, m->stream);
    if (r == HIPFFT_SUCCESS) r = hipfftSetStream(sp->inv, m->stream);
    if (r != HIPFFT_SUCCESS) {
        spectral_release(m);
        return fft_fail(r, "hipfftSetStream");
    }
    const double two_pi = 2.0 * M_PI;
    sp->args.uh = sp->uh;
    sp->args.nh = sp->nh;
    sp->args.nxh = nxh;
    sp->args.ny = ny;
    sp->args.nz = nz;
    sp->args.sx = two_pi / ((double)nx * d.dx);
    sp->args.sy = two_pi / ((double)ny * d.dx);
    sp->args.sz = two_pi / ((double)nz * d.dx);
    sp->args.dt = d.dt;
    sp->args.inv_n = 1.0 / ((double)nx * (double)ny * (double)nz);
    return PF_OK;
}

pf_status spectral_step(Model *m, int par, const void *step_args)
{
    Spectral *sp = static_cast<Spectral *>(m->spec);
    if (!sp) return fail(PF_ERR_STATE, "spectral plans are missing");
    void *u = m->buf[0][par], *out = m->buf[0][par ^ 1];
    const bool fresh = sp->kept_par != par;
    sp->kept_par = -1;  // until this step completes
    hipError_t e = launch_spectral_nonlinear(m->L, step_args, out, m->stream);
    if (e != hipSuccess) return hip_fail(e, "spectral nonlinear launch");
    hipfftResult r = HIPFFT_SUCCESS;
    if (m->fp32) {
        if (fresh)
            r = hipfftExecR2C(sp->fwd, static_cast<hipfftReal *>(u), static_cast<hipfftComplex *>(sp->uh));
        if (r == HIPFFT_SUCCESS)
            r = hipfftExecR2C(sp->fwd, static_cast<hipfftReal *>(out), static_cast<hipfftComplex *>(sp->nh));
    } else {
        if (fresh)
            r = hipfftExecD2Z(sp->fwd, static_cast<hipfftDoubleReal *>(u),
                              static_cast<hipfftDoubleComplex *>(sp->uh));
        if (r == HIPFFT_SUCCESS)
            r = hipfftExecD2Z(sp->fwd, static_cast<hipfftDoubleReal *>(out),
                              static_cast<hipfftDoubleComplex *>(sp->nh));
    }
    if (r != HIPFFT_SUCCESS) return fft_fail(r, "forward transform");
    SpecArgs a = sp->args;
    a.u_scale = fresh ? a.inv_n : 1.0;
    e = launch_spectral_update(m->L, a, m->stream);
    if (e != hipSuccess) return hip_fail(e, "spectral update launch");
    if (m->fp32)
        r = hipfftExecC2R(sp->inv, static_cast<hipfftComplex *>(sp->nh), static_cast<hipfftReal *>(out));
    else
        r = hipfftExecZ2D(sp->inv, static_cast<hipfftDoubleComplex *>(sp->nh),
                          static_cast<hipfftDoubleReal *>(out));
    if (r != HIPFFT_SUCCESS) return fft_fail(r, "inverse transform");
    sp->kept_par = par ^ 1;
    return PF_OK;
}

}  // namespace pf
