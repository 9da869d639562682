"""MI355X (gfx950) semi-implicit anisotropic diffusion (Sharma & Hammett,
arXiv:1008.0861): a HIP library behind a C ABI (include/asd.h,
include/asd_extra.h) and its Python binding.

    from paper_1008_0861_amd import binding as asd
    g = asd.Grid((ny, nx), (hx, hy), bc="periodic", dtype=torch.float32)
    g.set_b(bx, by); g.set_field("T", T)
    g.step_semi_implicit(dt, nsteps)

The binding loads paper_1008_0861_amd/libasd.so (build it with
``python -m paper_1008_0861_amd.build``); there is no CPU fallback.
"""
