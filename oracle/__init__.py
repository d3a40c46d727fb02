"""FP64 CPU oracle of the diminished-reality inpainting path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may import this
package.  The product library never calls it: it shares no code, header, table or helper
with the GPU path, and it imports nothing from the product package.  Its only shared
dependency is ``drsynth`` (seeded synthetic inputs, which hold none of the method's
arithmetic).

Contents
--------
``network``  clip-mode forward: cut-out, token flags, patch embed, pre-LN window-attention
             blocks, final LN, transposed-conv decoder, composite.
``grad``     the training loss and its analytic FP64 gradient (reverse mode, by hand).
``stream``   stream mode: one new frame per call against cached K/V of past frames.
``prepost``  camera-resolution pre/post-processing: BGRA -> RGB, union + dilation of the
             selected instance masks, 2x downscale, nearest 2x upscale, u8 composite.

Parity status: every function is pinned by the ``-m "not gpu"`` tests (library routines,
brute force, closed forms, invariants, finite differences).  The paper prints no worked
numeric example of the network, so no value here is pinned to a number printed in the
paper itself.
"""
from . import network  # noqa: F401
