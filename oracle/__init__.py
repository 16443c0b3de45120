"""CPU oracle for the RGB-D GMM and PBAS classify-and-update step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of the method in numpy, used to check the GPU library.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path (the HIP library and its Python
binding) never imports, links or calls anything here, and this package never
imports the product path: the two share no code.  The only common input is
the synthetic scene generator in ``synth/``, which holds none of the method's
arithmetic.

Modules
-------
``depth``     depth uint16 -> 8-bit code (Sec. 4.2)
``philox``    Philox4x32-10 counter-based generator (Salmon et al., SC'11)
``gmm``       RGB-D Gaussian mixture model step (Sec. 3.1)
``pbas``      RGB-D Pixel-Based Adaptive Segmenter step (Sec. 3.2)
``metrics``   PWC / FNR / FPR / Si quality indicators (Sec. 5)
``postfilter`` median post-filter of a binary mask (base PBAS method's smoothing)
``static``    static-object detection on a mask sequence (reading of Sec. 6's future work)

Floating point follows IEEE binary32 (or binary64 for the gradient reference)
with every operation rounded separately, in the order written in each
function; numpy never fuses a multiply and an add.
"""
