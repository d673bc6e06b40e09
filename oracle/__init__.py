"""CPU oracle for the LoD strand-hair rendering path (arxiv 2405.10565).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its Python
binding) may import, call or link anything under this package; only the tests, the smoke
check and the benchmark's CPU-baseline leg use it.  It shares no code with the HIP path.

It is a plain, slow, deliberately unoptimised restatement of what the renderer computes:

  * fiber.py     single-fibre scattering function, near-field R/TT/TRT     (Sec. 3.1, 3.2)
  * aggregate.py the aggregated thick-hair scattering function             (Sec. 4)
  * rttd.py      the R / TT / D single-fibre model and its aggregated form   (Sec. 3.1, 4)
  * raster.py    projection, tile binning, coverage, alpha, depth key      (Sec. 5.2 strips)
  * lod.py       thick-hair (elliptical cluster) construction              (Sec. 5.1 step 3)
  * render.py    per-fragment radiance and depth-ordered compositing        (Sec. 3 eq. for L_o)
  * grad.py      gradient of the LoD fitting loss by torch autograd         (Sec. 4 quantities)

Precision: scattering, alpha, radiance and compositing are float64 (torch CPU).  The steps
whose float result decides an integer (projection and 1/16-pixel snapping, the half-width
that sets the coverage radius, the depth key that orders fragments) are evaluated in
float32 with a fixed operation order, the precision the GPU kernel takes those decisions in.

Parity pins: every function is pinned in tests/test_oracle_*.py against closed forms,
brute force or invariants.  The absolute appearance against the paper's images is
"parity unpinned": the paper prints no worked numeric example and its images are absent.
"""
