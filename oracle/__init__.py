"""FP64 CPU oracle for the sine/cosine-basis PSTD method (Wise, Jaros, Cox & Treeby, arXiv:2005.00322).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, links or runs this package: only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may use it.  It shares no code,
tables or constants with the HIP library under ``paper_2005_00322_amd/``; the only module both sides
use is ``workloads`` (seeded synthetic inputs, none of the method's arithmetic).

Contents
--------
``dtt``       the eight group I/II discrete trigonometric transforms as dense matrices built from their
              cosine/sine sums (FFTW's unnormalised convention, §3.2) and the inverse pairing of
              Eq. (inverse_transforms).
``pstd``      per-axis boundary cases (Table transform_choices), the differentiation-plus-staggered
              interpolation recipe (appendix tables "Differentiation with staggered grids"), the
              staggered time step of Eq. (dtt_pstd_solution) and its 2D/3D form (§4.3), energy,
              the discrete modal closed form and the reflection-coefficient combination of §5.
``images``    image-source solutions (§1, §5) with the leapfrog's own dispersion relation: an
              independent closed form that involves no transform at all.
``nop``       FP64 reference of the DCT-basis neural-operator surrogate (not in the paper).

Everything is float64 NumPy.  Speed is not a goal; each function follows the paper's steps in order.
"""
