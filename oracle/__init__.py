"""FP64 CPU oracle for the sampled-frame pixel stage.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, calls or links anything
here, and this package imports nothing from the product path.

Plain, slow, obviously correct implementations, each citing the passage of
Poms et al., "Scanner: Efficient Video Analysis at Scale" (SIGGRAPH 2018) it
follows, or the textbook method where the paper names none:

* sampling.py  -- stride / gather / range sampling and stencil-after-sampling
                  pairs (Sec. 3.2 "Sampling/spacing" and "Stencil" operations,
                  "Slicing"; Sec. 5.1.1 access patterns).
* color.py     -- NV12 -> RGB BT.601 in Q14 fixed point (the format conversion
                  that Sec. 4.3 calls decoder post-processing), bilinear Q8
                  resize (the Resize map of Sec. 3.1), 16-bin-per-channel HIST
                  (Sec. 5.1.2).
* hs.py        -- pyramidal Horn-Schunck optical flow (Horn & Schunck 1981),
                  the FLOW stencil S[0,1] of Sec. 3.2 on sampled frames.
* surrogate.py -- the BF16 conv encoder-decoder flow surrogate, its backward
                  pass, loss, Adam, the residual gate and EPE.

Parity status of every function is listed in each module's header.
"""
