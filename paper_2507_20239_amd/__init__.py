"""MI355X (gfx950) hot path of Gaussian-splatting training: projection,
tile binning, front-to-back compositing and its adjoint, densification
statistics and split/clone/prune compaction, behind the C ABI of libgsmi.so.

Submodules: `gsmi` (ctypes binding of the C ABI), `autograd`
(GaussianRasterizer, a torch.autograd.Function wrapper), `autotune` (batch
and persistent-grid tuning of the batched step), `synth` (seeded synthetic
inputs), `build` (hipcc build of libgsmi.so).
"""
__version__ = "0.1.0"
