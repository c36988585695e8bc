"""FP64 CPU oracle for the persistence-diagram Sinkhorn path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never calls it, and it shares no code with the GPU library: the only
common dependency is the seeded input generator package ``pdgen``, which
holds no transport arithmetic.

What it computes (Lacombe, Cuturi, Oudot, NeurIPS 2018):

* ``ground``      - discretisation of a diagram to a d x d histogram plus the
                    diagonal bin (section 3, "Discretization"), the dense
                    (d^2+1) x (d^2+1) cost C and kernel K (section 3,
                    "Convolutions"), and the 1-D tables k, m, k_Delta, m_Delta.
* ``sinkhorn``    - Algorithm 1: alternating Sinkhorn scaling on the dense
                    ground space, marginal-error stopping (eq. for
                    dist(P, Pi(a,b)) in section 3), Sinkhorn cost <P, C>.
* ``separable``   - Propositions 2 and 3 written out (separable K apply and
                    separable transport cost); used only to pin the dense
                    path against the paper's identities.
* ``matching``    - Proposition 1 ground truth: brute-force partial matchings
                    (the d_p definition, section 2) and the augmented
                    assignment problem of the proof of Proposition 1.
* ``barycenter``  - Algorithm 2 (multiplicative gradient update with the
                    gradient of Proposition 5).
* ``kmeans``      - section 5 k-means: assignment by Algorithm 1, centroids
                    by Algorithm 2.
* ``bounds``      - error control of section 3: the upper bound <R_t, C> of
                    the rounded plan (rounding algorithm of the supplementary
                    material, Proposition 4) and the c-transform lower bound.

Every function that has no pin to something other than itself says
"parity unpinned" in its docstring.
"""
from . import ground, sinkhorn, separable, matching, barycenter, kmeans  # noqa: F401
