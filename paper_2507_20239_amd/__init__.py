"""MI355X (gfx950) hot path of Gaussian-splatting training: projection,
tile binning, front-to-back compositing and its adjoint, densification
statistics and split/clone/prune compaction, behind the C ABI of libgsmi.so.

Submodules: `gsmi` (ctypes binding of the C ABI), `autograd`
(torch.autograd.Function wrapper), `schedule` (coarse-to-fine and
global-to-local schedules), `synth` (seeded synthetic inputs), `build`
(hipcc build of libgsmi.so).
"""
__version__ = "0.1.0"
