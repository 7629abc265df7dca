"""Plain FP64 CPU oracle for the Ginnungagap initial-conditions hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code,
headers, tables or constant generators with the HIP library; the two meet only
through the seeded input generators in ``tests/inputs.py``.

What it computes (arxiv 2511.10353, Sec. 2.1-2.2):

* ``noise``      - white noise W(x): i.i.d. N(0,1) per lattice cell (Sec. 2 step 1),
                   realised as Philox-4x32-10 counters + Box-Muller (see
                   ``philox.py`` and ``normal.py`` for the exact definition).
* ``cosmology``  - P(k) (BBKS transfer function, sigma_8 normalisation,
                   Einstein-de Sitter growth) and the velocity factor a H f.
* ``pipeline``   - Eq. (1) delta~ = sqrt(P) W~, Eq. (2) v~_j = i delta~ k_j/k^2,
                   the inverse transforms and Eq. (3) (Zel'dovich positions).

Everything is evaluated in float64 with numpy / scipy.fft, step by step in the
order the paper states, with no blocking or fusion.  Each module header lists
how its functions are pinned by the ``-m "not gpu"`` tests.
"""
