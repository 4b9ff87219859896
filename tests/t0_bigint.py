"""Pure-Python big-integer brute force for tiny rings (pins for the oracle).

Independent of the oracle: Python integers only, definitions written out
directly (O(N^2) evaluation, schoolbook negacyclic product, CRT).
"""


def brv(x, logn):
    r = 0
    for _ in range(logn):
        r = (r << 1) | (x & 1)
        x >>= 1
    return r


def ntt_definition(a, q, psi):
    """out[j] = a(psi^(2 brv(j) + 1)) by direct evaluation."""
    n = len(a)
    logn = n.bit_length() - 1
    out = []
    for j in range(n):
        x = pow(psi, 2 * brv(j, logn) + 1, q)
        acc, xp = 0, 1
        for k in range(n):
            acc = (acc + a[k] * xp) % q
            xp = xp * x % q
        out.append(acc)
    return out


def negacyclic_mul(a, b, q):
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                c[k] = (c[k] + a[i] * b[j]) % q
            else:
                c[k - n] = (c[k - n] - a[i] * b[j]) % q
    return c


def automorph(a, g, q):
    """a(X^g) mod X^N + 1 in coefficient form."""
    n = len(a)
    out = [0] * n
    for k in range(n):
        e = g * k % (2 * n)
        if e < n:
            out[e] = (out[e] + a[k]) % q
        else:
            out[e - n] = (out[e - n] - a[k]) % q
    return out


def crt(residues, moduli):
    """Integer in [0, prod(moduli)) with the given residues."""
    M = 1
    for m in moduli:
        M *= m
    x = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % M, M


def is_prime(n):
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True
