"""MI355X-native differentiable Gaussian-splat rasterizer and 3DGS registration.

The compute path is the HIP library `libloopsplat.so` (built in-tree from
`csrc/`); `lib` loads it lazily and raises if it is missing, so importing the
package (e.g. for `synth`) never needs a GPU.
"""

__all__ = ["synth", "lib", "render", "register", "serve"]
