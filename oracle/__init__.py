"""FP64 CPU oracle for batched optimal clip alignment (TEST INFRASTRUCTURE).

This package is a plain, slow, obviously-correct restatement of what the
alignment path computes, written from the paper (Sections 2.2, 3.1-3.3,
Eqs. 1-9).  It exists to check the GPU library: only the test suite, the
smoke entry and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the HIP path; its only common dependency is the seeded
input generator ``clipgen``, which holds none of the method's arithmetic.

Modules
-------
raster  -- clip model (Eq. 1): half-open rectangle rasterisation, 4-connected
           polygons and their bounding boxes.
cosine  -- cosine track: spectra, whitening, phase-correlation surface
           (Eqs. 3-5), masked argmax with the tie rule, cosine score and
           thresholded bit (Eq. 2).
edge    -- edge track: polygon correspondence (Sec. 2.2.2) and the separable
           L-infinity Min-Max midpoint solve (Eq. 6).
contour -- edge track over full boundary edges: contour tracing, canonical
           edge order, descriptor equality, and the topological-hash
           pre-filter (Sec. 2.2.2; Sec. 3.1 stage 1).
xcorr   -- the exact objective: the window shift with the largest overlap
           count (Sec. 3.2).
xysep   -- cosine track aligned by XY-separation interval competition
           (Sec. 3.2.1(2)) instead of phase correlation.
prune   -- safe pre-screening bounds (area, row/column signatures, polygon
           bounding-box sizes).
scp     -- surprisal-based greedy set cover, eager and lazy (Eqs. 7-9).
loop    -- coarse-to-fine closed loop with orphan re-injection (Sec. 3.1).
serve   -- best covering representative per arriving clip (Sec. 3.1 step 3
           applied to a fixed library).
cover   -- drivers that run the above over pair lists.

Readings of the paper where it is silent or ambiguous are fixed in the
module docstrings; every function names the passage it follows.
"""
