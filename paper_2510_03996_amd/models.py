"""Layer chains of the two served model shapes, built on the C ABI.

* LeNet-5-shaped stack at N=2^14 (8 limbs): conv 5x5 1->6 (generic
  schedule) -> degree-4 polynomial ReLU -> 2x2 average pooling, stride 2.
* ResNet-20-shaped chain at N=2^16 (24 limbs): conv 3x3 16->16 (special
  schedule on a replicated 16x32x32 input) -> conv 3x3 16->32 stride 2 ->
  global average pooling -> fully connected 64->10.

The layer shapes follow the paper's architecture tables (LeNet-5 and
ResNet-20 first stages); weights enter as plaintexts prepared by the model
owner (preloaded, resident in HBM).  A chain is a list of stages
``stage(ct, stream) -> ct`` that enqueue one layer each.
"""
from . import he

RELU4 = [15.0 / 256.0, 0.5, 105.0 / 128.0, 0.0, -105.0 / 256.0]


class Chain:
    def __init__(self, ctx, stages, keys, n_pts, levels, relin=False):
        self.ctx, self.stages, self.keys, self.n_pts, self.levels, self.relin = ctx, stages, keys, n_pts, levels, relin


def lenet_plan(ctx):
    fm0 = he.fmap(1, 28, 28)
    pc = ctx.conv2d_plan(fm0, 6, 5, 1, 0)
    pp = ctx.avgpool_plan(pc.out, 2, 2)
    keys = sorted(set(pc.keys()) | set(pp.keys()))
    return fm0, pc, pp, keys


def lenet_chain(ctx, kern_pts, pool_pts, delta):
    """kern_pts: 150 conv plaintexts; pool_pts: pooling compaction masks."""
    fm0, pc, pp, keys = lenet_plan(ctx)
    assert len(kern_pts) == pc.n_kernel_pts and len(pool_pts) == pp.n_mask_pts
    fm1 = pc.out
    stages = [
        lambda ct, s: ctx.conv2d(ct, fm0, 6, 5, 1, 0, kern_pts, [], stream=s)[0],
        lambda ct, s: ctx.poly4(ct, RELU4, delta, stream=s),
        lambda ct, s: ctx.avgpool(ct, fm1, 2, 2, pool_pts, stream=s)[0],
    ]
    return Chain(ctx, stages, keys, (pc.n_kernel_pts, pp.n_mask_pts), pc.levels + 3 + pp.levels, relin=True)


def lenet_vectors(conv_weights, mask_chains=he.CHAIN_HORNER, log_n=14):
    """The real slot vectors of the LeNet-shaped stack from the library's
    plaintext recipes (he_layer_plaintexts), in the order lenet_chain takes
    them: conv 5x5 1->6 kernel vectors (conv_weights [6][1][5][5]) and the
    2x2 / stride-2 pooling masks.  The model owner encodes them (CKKS
    encoding at the input level and the working scale) into kern_pts and
    pool_pts."""
    fm0 = he.fmap(1, 28, 28)
    kern = he.layer_plaintexts(he.LAYER_CONV, log_n, conv_weights, fm=fm0, out_ch=6, kernel=5, stride=1, padding=0,
                               mask_chains=mask_chains)
    fm1 = he.fmap(6, 24, 24, rs=28, cs=28 * 28)
    pool = he.layer_plaintexts(he.LAYER_AVGPOOL, log_n, fm=fm1, kernel=2, stride=2, mask_chains=mask_chains)
    return kern, pool


def resnet_vectors(wa, wb, wfc, mask_chains=he.CHAIN_HORNER, fc_form=he.FC_ROWS, log_n=16):
    """The real slot vectors of the ResNet-shaped chain, in the order
    resnet_chain takes them: conv A (wa [16][16][3][3]) kernel vectors and
    masks, conv B (wb [32][16][3][3]) kernel vectors and masks, the global
    pooling masks, the FC (wfc [10][64]) weight vectors and masks."""
    slots = (1 << log_n) // 2
    fm0 = he.fmap(16, 32, 32, reps=2)
    va = he.layer_plaintexts(he.LAYER_CONV, log_n, wa, fm=fm0, out_ch=16, kernel=3, stride=1, padding=1,
                             mask_chains=mask_chains)
    fa = he.fmap(16, 32, 32, reps=2 if 2 * 16 * 32 * 32 == slots else 1)
    vb = he.layer_plaintexts(he.LAYER_CONV, log_n, wb, fm=fa, out_ch=32, kernel=3, stride=2, padding=1,
                             mask_chains=mask_chains)
    fb = he.fmap(32, 16, 16)
    vg = he.layer_plaintexts(he.LAYER_AVGPOOL, log_n, fm=fb, kernel=0, stride=1, mask_chains=mask_chains)
    vf = he.layer_plaintexts(he.LAYER_FC, log_n, wfc, n_in=64, n_out=10, fc_form=fc_form)
    na, nb = 9 * 16, 9 * 32
    nf = 64 if fc_form == he.FC_DIAG else 10
    return (va[:na], va[na:], vb[:nb], vb[nb:], vg, vf[:nf], vf[nf:])


def resnet_plan(ctx):
    fm0 = he.fmap(16, 32, 32, reps=2)
    pa = ctx.conv2d_plan(fm0, 16, 3, 1, 1)
    pb = ctx.conv2d_plan(pa.out, 32, 3, 2, 1)
    pg = ctx.avgpool_plan(pb.out, 0, 1)
    pf = ctx.fc_plan(64, 10)
    keys = sorted(set(pa.keys()) | set(pb.keys()) | set(pg.keys()) | set(pf.keys()))
    return fm0, pa, pb, pg, pf, keys


def resnet_chain(ctx, a_kern, a_mask, b_kern, b_mask, gap_mask, fc_rows, fc_mask):
    fm0, pa, pb, pg, pf, keys = resnet_plan(ctx)
    fa, fb = pa.out, pb.out
    stages = [
        lambda ct, s: ctx.conv2d(ct, fm0, 16, 3, 1, 1, a_kern, a_mask, stream=s)[0],
        lambda ct, s: ctx.conv2d(ct, fa, 32, 3, 2, 1, b_kern, b_mask, stream=s)[0],
        lambda ct, s: ctx.avgpool(ct, fb, 0, 1, gap_mask, stream=s)[0],
        lambda ct, s: ctx.fc(ct, 64, 10, fc_rows, fc_mask, stream=s),
    ]
    counts = [(pa.n_kernel_pts, pa.n_mask_pts), (pb.n_kernel_pts, pb.n_mask_pts), (0, pg.n_mask_pts),
              (pf.n_kernel_pts, pf.n_mask_pts)]
    return Chain(ctx, stages, keys, counts, pa.levels + pb.levels + pg.levels + pf.levels)
