"""Host-side replay of the forward kernels' addressing (no GPU).

For every log psi shape of the GPU parity suite (the two cases that are kept off
the GPU included) and for the benchmark's launch configurations, this replays,
on the CPU, the index arithmetic of the forward kernels for every workgroup,
lane, column, row and layer of every launch of psr_logpsi / psr_local_energy:
the packed-spin words, the row frontier (global or LDS), the units-split
kernel's staging copy and residual reads, the per-site log p and the log psi
outputs.  It asserts that each access lies inside the buffer the library sizes
for it.  The launch layout (columns and sequences per workgroup, tiles per
wave, frontier placement, launch size, frontier bytes per sequence) is the
library's own, from psr_forward_shape; the per-lane arithmetic is the kernels'
(psr_fwd.hip, psr_fwd_split.hip), restated here.
"""

import math

import pytest

K_LDS_FRONTIER = 112 * 1024   # the lane-owns-all-units kernel's LDS frontier area (bytes)


@pytest.fixture(scope="module")
def P():
    import paper_2605_13807_amd as P  # noqa: N813
    P.lib()
    return P


def _launches(B, chunk):
    q = 0
    while q < B:
        n = min(chunk, B - q)
        yield q, n
        q += n


def _replay_kernel1(lx, ly, nl, d, B, sh):
    """fwd_kernel (psr_fwd.hip): lanes own every unit of NTC columns each."""
    ntc, waves, seqs = sh["ntc"], sh["waves"], sh["seqs"]
    chunk, fsb, lds = sh["launch_seqs"], sh["frontier_seq_bytes"], sh["lds_frontier"]
    N = lx * ly
    words = (N + 31) // 32
    ELT, slots = 4, d // 4
    pitch, zoff = d * ELT + 16, d * ELT
    cols = waves * ntc * 16
    front_bytes = chunk * fsb
    if lds:
        assert (zoff + seqs * nl * lx * pitch) <= K_LDS_FRONTIER
    for q_begin, q_count in _launches(B, chunk):
        q_end = q_begin + q_count
        for blk in range(math.ceil(q_count / seqs)):
            q0 = q_begin + blk * seqs
            if q0 >= q_end:
                continue
            for col in range(cols):
                k, t = divmod(col, lx)
                q = q0 + k
                valid = k < seqs and q < q_end
                srow = q if valid else q0
                assert 0 <= srow < B
                sl = (q0 + k - q_begin) if valid else 0
                assert 0 <= sl < chunk
                for j in range(ly):
                    i = lx - 1 - t if j & 1 else t
                    assert 0 <= i < lx
                    if valid:
                        ih = i + 1 if j & 1 else i - 1
                        sites = [j * lx + i] + ([j * lx + ih] if 0 <= ih < lx else []) + ([(j - 1) * lx + i] if j else [])
                        for site in sites:
                            assert 0 <= site < N and (site >> 5) < words
                        assert 0 <= q * N + j * lx + i < B * N          # log p per site
                    for g in range(4):
                        if lds:
                            base = zoff + ((k if valid else 0) * nl * lx + i) * pitch + g * slots * ELT
                            assert base + (nl - 1) * lx * pitch + slots * ELT <= K_LDS_FRONTIER
                        else:
                            base = ((sl * nl * lx + i) * d + g * slots) * ELT
                            assert base + (nl - 1) * lx * d * ELT + slots * ELT <= front_bytes
            # per-sequence sums: red[k lx + t] and the outputs
            for k in range(seqs):
                if q0 + k < q_end:
                    assert (k + 1) * lx <= cols and q0 + k < B


def _replay_kernel2(lx, ly, nl, d, B, sh):
    """fwd_split_kernel (psr_fwd_split.hip): waves split the units, share the columns."""
    ntc, seqs = sh["ntc"], sh["seqs"]
    chunk, fsb = sh["launch_seqs"], sh["frontier_seq_bytes"]
    C = 16 * ntc
    N = lx * ly
    words = (N + 31) // 32
    pitch = 4 * d + 16
    lbytes = lx * d * 4
    assert fsb == nl * lbytes
    front_bytes = chunk * fsb
    nkb, nt = d // 32, d // 16
    for q_begin, q_count in _launches(B, chunk):
        q_end = q_begin + q_count
        for blk in range(math.ceil(q_count / seqs)):
            q0 = q_begin + blk * seqs
            if q0 >= q_end:
                continue
            wbase = (q0 - q_begin) * nl * lbytes        # this workgroup's frontier
            rsrc = seqs * nl * lbytes                   # the buffer resource's range
            # the staging copy of each layer
            pieces = 4 * d // 16
            for col in range(seqs * lx):
                k, t = divmod(col, lx)
                if q0 + k >= q_end:
                    continue
                row = (col % ntc) * 16 + col // ntc
                assert row < C
                for j in range(1, ly):
                    i = lx - 1 - t if j & 1 else t
                    for l in range(nl):
                        src = (k * nl + l) * lbytes + i * 4 * d + (pieces - 1) * 16
                        assert src + 16 <= rsrc and wbase + src + 16 <= front_bytes
                assert row * pitch + pieces * 16 <= C * pitch
            for r16 in range(16):
                for c in range(ntc):
                    col = r16 * ntc + c
                    k, t = divmod(col, lx)
                    q = q0 + k
                    valid = k < seqs and q < q_end
                    kl = k if valid else 0
                    assert (c * 16 + r16) < C
                    for j in range(ly):
                        i = lx - 1 - t if j & 1 else t
                        if valid:
                            for site in (j * lx + i, (j - 1) * lx + i if j else j * lx + i):
                                assert 0 <= site < N and (site >> 5) < words
                            assert q * N + j * lx + i < B * N
                        for g in range(4):
                            fro = kl * nl * lbytes + i * 4 * d + g * d
                            for l in range(nl):
                                # frontier write (valid columns) and residual reads of the wave's tiles
                                last = fro + l * lbytes + ((nt - 1) >> 1) * 32 + 8 + 16 + 8
                                assert last <= rsrc and wbase + last <= front_bytes
                                assert fro + l * lbytes + (nkb - 1) * 32 + 32 <= rsrc


SHAPES = [
    # geom, lx, ly, nl, d, prec, B  (the log psi cases of the GPU parity suite)
    (0, 16, 1, 1, 32, 0, 512), (0, 16, 1, 1, 32, 1, 77), (1, 4, 4, 3, 32, 0, 100),
    (1, 5, 3, 2, 64, 0, 61),       # kept off the GPU after one fault
    (1, 10, 10, 2, 64, 0, 200), (1, 10, 10, 2, 64, 1, 200), (1, 4, 4, 3, 32, 1, 100), (1, 6, 5, 2, 64, 1, 50),
    (1, 8, 8, 3, 128, 1, 20), (1, 1, 7, 2, 32, 0, 33),
    (1, 9, 1, 3, 32, 0, 33),       # kept off the GPU after one fault
    (1, 20, 20, 3, 128, 0, 24), (1, 20, 20, 3, 128, 1, 24), (1, 32, 32, 3, 128, 0, 9), (1, 32, 32, 3, 128, 1, 9),
    (1, 52, 52, 4, 256, 0, 2), (1, 52, 52, 4, 256, 1, 2), (1, 60, 3, 4, 256, 1, 3), (1, 64, 2, 2, 64, 1, 5),
    (1, 16, 3, 2, 256, 1, 4), (1, 4, 4, 3, 32, 2, 100), (1, 10, 10, 2, 64, 2, 200), (1, 20, 20, 3, 128, 2, 24),
    (1, 32, 32, 3, 128, 2, 9), (1, 52, 52, 4, 256, 2, 2), (1, 60, 3, 4, 256, 2, 3), (1, 64, 2, 2, 64, 2, 5),
    (1, 40, 3, 3, 256, 1, 7), (1, 13, 5, 2, 256, 2, 23), (1, 20, 4, 3, 128, 2, 11), (1, 64, 2, 3, 128, 1, 3),
]


@pytest.mark.parametrize("geom,lx,ly,nl,d,prec,B", SHAPES)
def test_forward_addressing_in_bounds(P, geom, lx, ly, nl, d, prec, B):
    m = P.Model(geom, lx, ly, nl, d, prec)
    sh = P.forward_shape(m, B)
    assert sh["seqs"] >= 1 and sh["cols"] == sh["waves"] * sh["ntc"] * 16 if not sh["split_kernel"] else True
    if sh["split_kernel"]:
        _replay_kernel2(lx, ly, nl, d, B, sh)
    else:
        _replay_kernel1(lx, ly, nl, d, B, sh)


@pytest.mark.parametrize("L,nl,d,prec,chunk,n_seq", [(52, 4, 256, 1, 32768, 70000), (32, 3, 128, 1, 32768, 40000),
                                                     (10, 2, 64, 0, 1000, 2500)])
def test_eloc_launch_configuration_in_bounds(P, L, nl, d, prec, chunk, n_seq):
    """The connected-configuration launches of psr_local_energy (chunks of `chunk`
    sequences against a frontier of `chunk` sequences), with a ragged last chunk."""
    m = P.Model(1, L, L, nl, d, prec)
    sh = dict(P.forward_shape(m, 1))
    sh["launch_seqs"] = chunk
    if sh["split_kernel"]:
        _replay_kernel2_sampled(L, nl, d, n_seq, sh)
    else:
        _replay_kernel1(L, L, nl, d, n_seq, sh)


def _replay_kernel2_sampled(L, nl, d, n_seq, sh):
    """The units-split kernel over n_seq sequences in launches of sh['launch_seqs']: the
    workgroups of each launch's first and last blocks (the only ones whose offsets can
    approach the frontier's end or the launch's end)."""
    seqs, chunk = sh["seqs"], sh["launch_seqs"]
    for q_begin, q_count in _launches(n_seq, chunk):
        blocks = math.ceil(q_count / seqs)
        for blk in {0, blocks - 1}:
            sub = dict(sh)
            # replay one block as a launch of its own sequences, inside the full frontier
            q0 = blk * seqs
            n = min(seqs, q_count - q0)
            front = chunk * sh["frontier_seq_bytes"]
            lbytes = L * d * 4
            assert (q0 + n) * nl * lbytes <= front
            sub["launch_seqs"] = n
            _replay_kernel2(L, L, nl, d, n, sub)
