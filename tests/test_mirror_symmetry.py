"""The mirror symmetry the three-step kernel's mirror mode relies on, and the
index rules of that mode, checked on the CPU.

Swapping the forward and backward path of every point (Liouville digit
(a, b) -> (b, a)) maps the path sum of Sec. II to its complex conjugate when
rho(0) is Hermitian: K = U (x) U* and every influence factor
exp(-(s_a - s_b)(eta s_c - eta* s_d)) go to their conjugates.  So the tensor
entry at the mirrored index is the conjugate of the entry.  The first tests
pin that on the brute-force path sum (oracle, independent of the kernel);
the others model which items the mirror-mode launches run, which entries
they store where, and how rho is formed from the items that run.
"""
import numpy as np
import pytest

from oracle import brute, run
from paper_1205_6872_amd import workloads as W


def mirror4(x):
    """Each base-4 digit o = 2a + b -> 2b + a (the kernel's bit form)."""
    x = np.asarray(x, dtype=np.int64)
    return ((x & 0x5555555555555555) << 1) | ((x >> 1) & 0x5555555555555555)


def mirror_by_digits(x, n_digits):
    out = 0
    for j in range(n_digits):
        d = (x // 4 ** j) % 4
        a, b = d // 2, d % 2
        out += (2 * b + a) * 4 ** j
    return out


def _hermitian_rho0(rng):
    r = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    r = r @ r.conj().T
    return r / np.trace(r)


def _brute(w, n):
    inp = run.inputs_from(w)
    Gf = run.G_function(inp)
    _, _, _, K = run.setup(inp)
    return brute.brute_tensor(inp.s, K, inp.rho0, Gf, inp.dt, inp.L, n)


def test_bit_form_is_the_digit_swap():
    xs = np.arange(4 ** 6)
    assert np.array_equal(mirror4(xs), [mirror_by_digits(int(x), 6) for x in xs])
    assert np.array_equal(mirror4(mirror4(xs)), xs)


@pytest.mark.parametrize("seed,L,n", [(1, 3, 5), (2, 4, 6), (3, 2, 5)])
def test_path_sum_entries_are_conjugate_under_the_mirror(seed, L, n):
    rng = np.random.default_rng(seed)
    w = W.spin_boson_l7().with_(L=L, H=W.random_hermitian(rng, 2), rho0=_hermitian_rho0(rng), xi=0.4)
    A = _brute(w, n)
    x = np.arange(len(A))
    scale = np.abs(A).max()
    assert np.abs(A[mirror4(x)] - np.conj(A)).max() <= 1e-14 * scale
    # not trivially so: the mirrored entries differ from the entries themselves
    assert np.abs(A[mirror4(x)] - A).max() > 1e-3 * scale


def test_a_non_hermitian_rho0_breaks_it():
    rng = np.random.default_rng(4)
    rho0 = np.array([[0.7, 0.2 + 0.1j], [0.05 - 0.3j, 0.3]])
    w = W.spin_boson_l7().with_(L=3, H=W.random_hermitian(rng, 2), rho0=rho0, xi=0.4)
    A = _brute(w, 5)
    x = np.arange(len(A))
    assert np.abs(A[mirror4(x)] - np.conj(A)).max() > 1e-3 * np.abs(A).max()


def _split(nd):
    """A digit split of nd item digits like the kernel's: low digits per
    thread, middle digits swept, the rest per block."""
    d_lo = min(2, nd)
    d_mid = min(2, nd - d_lo)
    return 4 ** d_lo, 4 ** d_mid, 4 ** (nd - d_lo - d_mid)


def diagonal_digits(x):
    """Bit i of x -> digit i = 3 (else 0), as the kernel forms the items whose
    digits are all diagonal."""
    out = 0
    i = 0
    while x:
        if x & 1:
            out += 3 * 4 ** i
        x >>= 1
        i += 1
    return out


def mirror_launches(R, Q, grid, block=256):
    """The items each mirror-mode launch runs, in the host's partition: mode 1
    one block per high-digit value below its mirror; mode 2 `parts` blocks per
    value equal to its mirror, q_span sweep rows each, items below their
    mirror; mode 3 one block per such value, the items equal to their mirror.
    Returns [(mode, partial row, item m)] and the number of partial rows."""
    canon = [h for h in range(grid) if h < mirror4(h)]
    diag = [h for h in range(grid) if h == mirror4(h)]
    rows_per_pass = block // R
    passes = (Q + rows_per_pass - 1) // rows_per_pass
    parts = max(1, min(passes, -(-256 // max(len(diag), 1))))
    span = ((passes + parts - 1) // parts) * rows_per_pass
    dl, dm = int(round(np.log(R) / np.log(4))), int(round(np.log(Q) / np.log(4)))
    runs = []
    for b, h in enumerate(canon):
        for q in range(Q):
            for r in range(R):
                runs.append((1, b, h * R * Q + q * R + r))
    for b in range(len(diag) * parts):
        h, part = diag[b // parts], b % parts
        for t in range(block):
            for q in range(part * span + t // R, min(Q, (part + 1) * span), rows_per_pass):
                m = h * R * Q + q * R + t % R
                if mirror4(m) > m:
                    runs.append((2, len(canon) + b, m))
    for b, h in enumerate(diag):
        for it in range(1 << (dl + dm)):
            r, q = diagonal_digits(it & ((1 << dl) - 1)), diagonal_digits(it >> dl)
            runs.append((3, len(canon) + len(diag) * parts + b, h * R * Q + q * R + r))
    return runs, len(canon) + len(diag) * (parts + 1)


@pytest.mark.parametrize("R,Q,grid", [(1, 1, 1), (4, 1, 1), (16, 4, 1), (64, 64, 1), (64, 64, 16),
                                      (16, 16, 64), (64, 16, 4), (256, 1, 16)])
def test_mirror_launches_run_each_kept_item_once(R, Q, grid):
    runs, n_rows = mirror_launches(R, Q, grid)
    items = [m for _, _, m in runs]
    n_items = R * Q * grid
    assert len(items) == len(set(items))
    assert set(items) == {m for m in range(n_items) if m <= mirror4(m)}
    assert all(mode == 3 for mode, _, m in runs if mirror4(m) == m)
    assert all(mode != 3 for mode, _, m in runs if mirror4(m) != m)
    assert max(row for _, row, _ in runs) < n_rows <= max(grid, 1) + (2 ** int(round(np.log(grid) / np.log(4)))) * 64


def pair_mirror_launches(R, Q, grid, block=256):
    """The items each mirror-mode launch of the two-step kernel runs, thread
    by thread as the kernel maps them: mode 1 every row of a block whose high
    digits are below their mirror; mode 2 the sweep rows of its part, items
    below their mirror; mode 3 the threads whose low digits are all diagonal,
    sweeping the diagonal middle digits.  Returns [(mode, partial row, item)]
    and the number of partial rows."""
    canon = [h for h in range(grid) if h < mirror4(h)]
    diag = [h for h in range(grid) if h == mirror4(h)]
    cols = block // R
    passes = (Q + cols - 1) // cols
    parts = max(1, min(passes, -(-256 // max(len(diag), 1))))
    span = ((passes + parts - 1) // parts) * cols
    dm = int(round(np.log(Q) / np.log(4)))
    runs = []
    for b, h in enumerate(canon):
        for t in range(cols * R):
            for q in range(t // R, Q, cols):
                runs.append((1, b, h * R * Q + q * R + t % R))
    for b in range(len(diag) * parts):
        h, part = diag[b // parts], b % parts
        for t in range(cols * R):
            for q in range(part * span + t // R, min(Q, (part + 1) * span), cols):
                m = h * R * Q + q * R + t % R
                if mirror4(m) > m:
                    runs.append((2, len(canon) + b, m))
    for b, h in enumerate(diag):
        for t in range(cols * R):
            r = t % R
            if mirror4(r) != r:                    # a low digit off the diagonal
                continue
            for it in range(t // R, 1 << dm, cols):
                runs.append((3, len(canon) + len(diag) * parts + b, h * R * Q + diagonal_digits(it) * R + r))
    return runs, len(canon) + len(diag) * (parts + 1)


@pytest.mark.parametrize("R,Q,grid", [(4, 1, 1), (16, 1, 1), (64, 1, 1), (64, 4, 1), (64, 16, 1), (64, 64, 1),
                                      (64, 64, 4), (64, 64, 64), (64, 16, 16)])
def test_pair_mirror_launches_run_each_kept_item_once(R, Q, grid):
    """The two-step kernel's split: R = 4^min(3, digits) low digits per
    thread, Q = 4^(0..3) middle digits swept, the rest per block."""
    runs, n_rows = pair_mirror_launches(R, Q, grid)
    items = [m for _, _, m in runs]
    assert len(items) == len(set(items))
    assert set(items) == {m for m in range(R * Q * grid) if m <= mirror4(m)}
    assert all(mode == 3 for mode, _, m in runs if mirror4(m) == m)
    assert all(mode != 3 for mode, _, m in runs if mirror4(m) != m)
    assert max(row for _, row, _ in runs) < n_rows


@pytest.mark.parametrize("width", [2, 3])
@pytest.mark.parametrize("nd", [0, 1, 3, 4, 5, 6])
def test_mirror_pass_index_rules(nd, width):
    """Items are m (nd digits) with E = 4^width entries each (the two- and
    three-step kernels).  Mode 1 runs the blocks
    whose high digits are below their mirror, with no per-item test; mode 2
    the blocks equal to their mirror, skipping items above their mirror.
    Input: only entries not above their mirror are valid.  Output: each item
    stores entry (m, c) if c is not above its mirror, else the conjugate at
    (mirror(m), mirror(c)) unless m is its own mirror."""
    rng = np.random.default_rng(nd)
    R, Q, grid = _split(nd)
    n_items = 4 ** nd
    E = 4 ** width
    entries = E * n_items
    x = np.arange(entries)
    keep = x <= mirror4(x)

    def symmetric(v):
        v = v.copy()
        up = x > mirror4(x)
        v[up] = np.conj(v[mirror4(x[up])])
        return v

    X = symmetric(rng.normal(size=entries) + 1j * rng.normal(size=entries))   # a valid input tensor
    Y = symmetric(rng.normal(size=entries) + 1j * rng.normal(size=entries))   # what a full step would write
    Xh = np.where(keep, X, np.nan)                                           # half-valid input
    # output layout: entry (m, c) at m + n_items * c
    out_index = (np.arange(n_items)[:, None] + n_items * np.arange(E)[None, :])
    Yc = Y[out_index]                                                        # Yc[m, c]
    assert np.array_equal(mirror4(out_index), out_index[mirror4(np.arange(n_items))][:, mirror4(np.arange(E))])

    out = np.full(entries, np.nan + 0j)
    writes = np.zeros(entries, dtype=int)
    # rho-like linear functional with mirror-covariant weights: W[mirror(o), mirror(c)] = conj(W[o, c])
    Wt = rng.normal(size=(4, E)) + 1j * rng.normal(size=(4, E))
    for o in range(4):
        for c in range(E):
            if (int(mirror4(o)), int(mirror4(c))) < (o, c):
                Wt[o, c] = np.conj(Wt[int(mirror4(o)), int(mirror4(c))])
            elif (int(mirror4(o)), int(mirror4(c))) == (o, c):
                Wt[o, c] = Wt[o, c].real
    rho_full = sum(Wt @ Yc[m] for m in range(n_items))
    rho_half = np.zeros(4, dtype=complex)

    ran = set()
    blocks = [(h, 1) for h in range(grid) if h < mirror4(h)] + [(h, 2) for h in range(grid) if h == mirror4(h)]
    assert len(blocks) == (grid + 2 ** int(round(np.log(grid) / np.log(4)))) // 2
    for h, mode in blocks:
        for q in range(Q):
            for r in range(R):
                m = h * R * Q + q * R + r
                mb = int(mirror4(m))
                if mode == 1:
                    assert m < mb                     # the no-per-item-test claim
                elif mb < m:
                    continue
                ran.add(m)
                self_m = m == mb
                w = Xh[E * m:E * m + E].copy()
                if self_m:
                    for k in range(E):
                        if mirror4(k) < k:
                            w[k] = np.conj(w[mirror4(k)])
                assert np.array_equal(w, X[E * m:E * m + E])      # every value the item uses is valid
                v = Wt @ Yc[m]
                if self_m:
                    rho_half += v
                else:
                    rho_half += v + np.conj(v[[0, 2, 1, 3]])
                for c in range(E):
                    cb = int(mirror4(c))
                    if cb >= c:
                        out[m + n_items * c] = Yc[m, c]
                        writes[m + n_items * c] += 1
                    elif not self_m:
                        out[mb + n_items * cb] = np.conj(Yc[m, c])
                        writes[mb + n_items * cb] += 1
    assert ran == {m for m in range(n_items) if m <= mirror4(m)}
    assert np.array_equal(writes, keep.astype(int))                      # every kept entry once, nothing else
    assert np.array_equal(out[keep], Y[keep])
    assert np.abs(rho_half - rho_full).max() <= 1e-9 * np.abs(rho_full).max()
    # completion: entries above their mirror take the conjugate of it
    up = ~keep
    out[up] = np.conj(out[mirror4(x[up])])
    assert np.array_equal(out, Y)


# ---------------------------------------------------------------- M = 4 (N = 16)
def mirror16(x):
    """Each base-16 digit o = 4a + b -> 4b + a (the kernel's bit form)."""
    x = np.asarray(x, dtype=np.int64)
    return ((x & 0x3333333333333333) << 2) | ((x >> 2) & 0x3333333333333333)


def test_bit_form_is_the_digit_swap_m4():
    xs = np.arange(16 ** 3)
    want = []
    for x in xs:
        out = 0
        for j in range(3):
            d = (int(x) // 16 ** j) % 16
            out += (4 * (d % 4) + d // 4) * 16 ** j
        want.append(out)
    assert np.array_equal(mirror16(xs), want)


def test_path_sum_entries_are_conjugate_under_the_mirror_m4():
    rng = np.random.default_rng(12)
    r = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    rho0 = r @ r.conj().T
    rho0 /= np.trace(rho0)
    w = W.spin_boson_l7().with_(M=4, s=np.linspace(-1, 1, 4), H=W.random_hermitian(rng, 4), rho0=rho0,
                                L=2, xi=0.3)
    A = _brute(w, 3)
    x = np.arange(len(A))
    scale = np.abs(A).max()
    assert np.abs(A[mirror16(x)] - np.conj(A)).max() <= 1e-14 * scale
    assert np.abs(A[mirror16(x)] - A).max() > 1e-3 * scale


def mfma_mirror_launches(Q, grid, waves=4):
    """Items run by the N = 16 MFMA step's mirror launches: 16 items per wave
    row (lane column j = the lowest digit), Q sweep rows over the block's
    `waves` waves; mode 1 the high-digit values below their mirror; mode 2
    the values equal to it, `parts` blocks of q_span rows, items below their
    mirror; mode 3 the same values, rows whose digits are all diagonal
    (base-4 digit d -> 5 d), lanes j with a diagonal digit."""
    canon = [h for h in range(grid) if h < mirror16(h)]
    diag = [h for h in range(grid) if h == mirror16(h)]
    passes = (Q + waves - 1) // waves
    parts = max(1, min(passes, -(-256 // max(len(diag), 1))))
    span = ((passes + parts - 1) // parts) * waves
    dm = int(round(np.log(Q) / np.log(16)))
    runs = []
    for b, h in enumerate(canon):
        for q in range(Q):
            for j in range(16):
                runs.append((1, b, h * 16 * Q + 16 * q + j))
    for b in range(len(diag) * parts):
        h, part = diag[b // parts], b % parts
        for wv in range(waves):
            for q in range(part * span + wv, min(Q, (part + 1) * span), waves):
                for j in range(16):
                    m = h * 16 * Q + 16 * q + j
                    if m < mirror16(m):
                        runs.append((2, len(canon) + b, m))
    for b, h in enumerate(diag):
        for it in range(4 ** dm):
            q = sum((5 * ((it >> (2 * k)) & 3)) << (4 * k) for k in range(dm))
            for j in range(0, 16, 5):
                runs.append((3, len(canon) + len(diag) * parts + b, h * 16 * Q + 16 * q + j))
    return runs, len(canon) + len(diag) * (parts + 1)


@pytest.mark.parametrize("Q,grid", [(1, 1), (16, 1), (1, 16), (16, 16), (256, 16), (16, 256)])
def test_mfma_mirror_launches_run_each_kept_item_once(Q, grid):
    runs, n_rows = mfma_mirror_launches(Q, grid)
    items = [m for _, _, m in runs]
    assert len(items) == len(set(items))
    assert set(items) == {m for m in range(16 * Q * grid) if m <= mirror16(m)}
    assert all(mode == 3 for mode, _, m in runs if mirror16(m) == m)
    assert all(mode != 3 for mode, _, m in runs if mirror16(m) != m)
    assert max(row for _, row, _ in runs) < n_rows


# ----------------------------------------------------------------- M = 3 (N = 9)
def mirror9(x):
    out, w = 0, 1
    x = int(x)
    while x > 0:
        d = x % 9
        out += (3 * (d % 3) + d // 3) * w
        x //= 9
        w *= 9
    return out


def test_path_sum_entries_are_conjugate_under_the_mirror_m3():
    rng = np.random.default_rng(13)
    r = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    rho0 = r @ r.conj().T
    rho0 /= np.trace(rho0)
    w = W.three_site_l8().with_(L=2, H=W.random_hermitian(rng, 3), rho0=rho0, xi=0.3)
    A = _brute(w, 3)
    mb = np.array([mirror9(x) for x in range(len(A))])
    scale = np.abs(A).max()
    assert np.abs(A[mb] - np.conj(A)).max() <= 1e-14 * scale
    assert np.abs(A[mb] - A).max() > 1e-3 * scale


def vector_mirror_launches(N, R, Q, grid, block=256):
    """Items run by the vector step's mirror launches (N = 4 or 9): thread
    columns r = t % R (block // R of them per row), Q sweep rows; mode 1 the
    high-digit values below their mirror; mode 2 those equal to it, `parts`
    blocks of q_span rows, items below their mirror; mode 3 the same values,
    threads whose low digits are all diagonal, rows whose digits are."""
    M = 2 if N == 4 else 3
    mir = (lambda x: int(mirror4(x))) if N == 4 else mirror9

    def diag_only(v):
        while v > 0:
            if v % N % (M + 1):
                return False
            v //= N
        return True

    def diag_digits(x):
        out, w = 0, 1
        while x > 0:
            out += (M + 1) * (x % M) * w
            x //= M
            w *= N
        return out

    canon = [h for h in range(grid) if h < mir(h)]
    diag = [h for h in range(grid) if h == mir(h)]
    cR = block // R
    passes = (Q + cR - 1) // cR
    parts = max(1, min(passes, -(-256 // max(len(diag), 1))))
    span = ((passes + parts - 1) // parts) * cR
    n_rows = 1
    q = Q
    while q > 1:
        n_rows *= M
        q //= N
    runs = []
    for b, h in enumerate(canon):
        for qm in range(Q):
            for r in range(R):
                runs.append((1, b, h * R * Q + qm * R + r))
    for b in range(len(diag) * parts):
        h, part = diag[b // parts], b % parts
        for t in range(cR * R):
            for qm in range(part * span + t // R, min(Q, (part + 1) * span), cR):
                m = h * R * Q + qm * R + t % R
                if m < mir(m):
                    runs.append((2, len(canon) + b, m))
    for b, h in enumerate(diag):
        for t in range(cR * R):
            if not diag_only(t % R):
                continue
            for it in range(t // R, n_rows, cR):
                runs.append((3, len(canon) + len(diag) * parts + b, h * R * Q + diag_digits(it) * R + t % R))
    return runs, len(canon) + len(diag) * (parts + 1), mir


@pytest.mark.parametrize("N,R,Q,grid", [(9, 1, 1, 1), (9, 9, 1, 1), (9, 81, 9, 1), (9, 81, 81, 9), (9, 9, 9, 81),
                                        (9, 81, 1, 729), (4, 1, 1, 1), (4, 4, 1, 1), (4, 256, 16, 4),
                                        (4, 256, 1, 64), (4, 64, 4, 16), (4, 256, 16, 256)])
def test_vector_mirror_launches_run_each_kept_item_once(N, R, Q, grid):
    runs, n_rows, mir = vector_mirror_launches(N, R, Q, grid)
    items = [m for _, _, m in runs]
    assert len(items) == len(set(items))
    assert set(items) == {m for m in range(R * Q * grid) if m <= mir(m)}
    assert all(mode == 3 for mode, _, m in runs if mir(m) == m)
    assert max(row for _, row, _ in runs) < n_rows
