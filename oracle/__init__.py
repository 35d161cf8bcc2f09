"""Plain FP64 CPU oracle for the Fast Cauchy Transform l1-regression hot path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call, link
or execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_1207_4684_amd``) and imports nothing from it.

It restates, slowly and plainly, what the method of Clarkson, Drineas,
Magdon-Ismail, Mahoney, Meng and Woodruff, "The Fast Cauchy Transform and
Faster Robust Linear Regression" (arXiv 1207.4684), computes on its
data-parallel path:

* ``philox``   -- the counter-based generator every random quantity is drawn
                  from (Salmon et al., SC'11), and the stream layout;
* ``fct``      -- FCT1, Pi1 = 4 B C H~ (Section "FCT1 Construction"), fast and
                  dense forms, and the normalized Sylvester Hadamard;
* ``basis``    -- QR of the sketch and M = R^-1 Pi2 (FastL1Basis figure; steps
                  2-4 of the FastCauchyRegression figure);
* ``sampling`` -- lambda_i = median_j |(X R^-1 Pi2)_ij|, p_i, the Bernoulli
                  sampling matrix D and the gathered coreset (steps 4-7);
* ``l1``       -- exact l1 optima (brute force over interpolating subsets,
                  linear programming as in step 8, a vertex certificate, a
                  weak-duality lower bound, weighted medians);
* ``pipeline`` -- the whole FastCauchyRegression path;
* ``lowp``     -- round-to-nearest-even BF16 rounding with integer operations.

Everything is FP64 unless the input bytes are of another type.  Functions
that are not pinned by an independent check say "parity unpinned".
"""
