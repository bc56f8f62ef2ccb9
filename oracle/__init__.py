"""CPU oracle for batch-dynamic subgraph matching.

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything from this package.  The
GPU library and its Python binding never import it, and it shares no code
with them; the seeded input generators in ``workloads`` are the only module
both sides use.

Contents
  brute         O1: complete enumeration of the matches of Q in G and in G',
                then their set differences (Def. 2 and the problem statement
                of Sec. II-A).
  plain         O2: the plain incremental enumerator (C, libo2.so) that
                follows Algorithm 1 of Sec. IV-C with the order rule stated
                after it; ctypes wrapper.
  vertices      vertex insertions and deletions reduced to edge updates
                (Sec. II-A), for use with brute and plain.
  closed_forms  closed-form counts (stars, single edges, equal-label
                triangles), label-preserving automorphisms, per-tuple
                validation and the multiset hash.
"""
