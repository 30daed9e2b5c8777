// Per-l_a dispatch tables of the k_tile instantiations (one translation unit
// per (la, lb) keeps the device compile parallel): tile_table_la<l_a>()[lb * 2 + D].
#include "shg_kernels.h"
namespace shg {
const tile_fn *tile_fns_la0_lb0();
const tile_fn *tile_fns_la0_lb1();
const tile_fn *tile_fns_la0_lb2();
const tile_fn *tile_fns_la0_lb3();
const tile_fn *tile_fns_la0_lb4();
const tile_fn *tile_fns_la1_lb0();
const tile_fn *tile_fns_la1_lb1();
const tile_fn *tile_fns_la1_lb2();
const tile_fn *tile_fns_la1_lb3();
const tile_fn *tile_fns_la1_lb4();
const tile_fn *tile_fns_la2_lb0();
const tile_fn *tile_fns_la2_lb1();
const tile_fn *tile_fns_la2_lb2();
const tile_fn *tile_fns_la2_lb3();
const tile_fn *tile_fns_la2_lb4();
const tile_fn *tile_fns_la3_lb0();
const tile_fn *tile_fns_la3_lb1();
const tile_fn *tile_fns_la3_lb2();
const tile_fn *tile_fns_la3_lb3();
const tile_fn *tile_fns_la3_lb4();
const tile_fn *tile_fns_la4_lb0();
const tile_fn *tile_fns_la4_lb1();
const tile_fn *tile_fns_la4_lb2();
const tile_fn *tile_fns_la4_lb3();
const tile_fn *tile_fns_la4_lb4();
const tile_fn *tile_fns_la5_lb0();
const tile_fn *tile_fns_la5_lb1();
const tile_fn *tile_fns_la5_lb2();
const tile_fn *tile_fns_la5_lb3();
const tile_fn *tile_fns_la6_lb0();
const tile_fn *tile_fns_la6_lb1();
const tile_fn *tile_fns_la6_lb2();
const tile_fn *tile_fns_la6_lb3();
const tile_fn *tile_fns_la7_lb0();
const tile_fn *tile_fns_la7_lb1();
const tile_fn *tile_fns_la7_lb2();
const tile_fn *tile_fns_la7_lb3();
const tile_fn *tile_fns_la8_lb0();
const tile_fn *tile_fns_la8_lb1();
const tile_fn *tile_fns_la8_lb2();
const tile_fn *tile_fns_la8_lb3();
const tile_fn *tile_fns_la9_lb0();
const tile_fn *tile_fns_la9_lb1();
const tile_fn *tile_fns_la9_lb2();
const tile_fn *tile_fns_la9_lb3();

const tile_fn *tile_table_la0()
{
    static const tile_fn t[] = {tile_fns_la0_lb0()[0], tile_fns_la0_lb0()[1], tile_fns_la0_lb1()[0], tile_fns_la0_lb1()[1], tile_fns_la0_lb2()[0], tile_fns_la0_lb2()[1], tile_fns_la0_lb3()[0], tile_fns_la0_lb3()[1], tile_fns_la0_lb4()[0], tile_fns_la0_lb4()[1]};
    return t;
}
const tile_fn *tile_table_la1()
{
    static const tile_fn t[] = {tile_fns_la1_lb0()[0], tile_fns_la1_lb0()[1], tile_fns_la1_lb1()[0], tile_fns_la1_lb1()[1], tile_fns_la1_lb2()[0], tile_fns_la1_lb2()[1], tile_fns_la1_lb3()[0], tile_fns_la1_lb3()[1], tile_fns_la1_lb4()[0], tile_fns_la1_lb4()[1]};
    return t;
}
const tile_fn *tile_table_la2()
{
    static const tile_fn t[] = {tile_fns_la2_lb0()[0], tile_fns_la2_lb0()[1], tile_fns_la2_lb1()[0], tile_fns_la2_lb1()[1], tile_fns_la2_lb2()[0], tile_fns_la2_lb2()[1], tile_fns_la2_lb3()[0], tile_fns_la2_lb3()[1], tile_fns_la2_lb4()[0], tile_fns_la2_lb4()[1]};
    return t;
}
const tile_fn *tile_table_la3()
{
    static const tile_fn t[] = {tile_fns_la3_lb0()[0], tile_fns_la3_lb0()[1], tile_fns_la3_lb1()[0], tile_fns_la3_lb1()[1], tile_fns_la3_lb2()[0], tile_fns_la3_lb2()[1], tile_fns_la3_lb3()[0], tile_fns_la3_lb3()[1], tile_fns_la3_lb4()[0], tile_fns_la3_lb4()[1]};
    return t;
}
const tile_fn *tile_table_la4()
{
    static const tile_fn t[] = {tile_fns_la4_lb0()[0], tile_fns_la4_lb0()[1], tile_fns_la4_lb1()[0], tile_fns_la4_lb1()[1], tile_fns_la4_lb2()[0], tile_fns_la4_lb2()[1], tile_fns_la4_lb3()[0], tile_fns_la4_lb3()[1], tile_fns_la4_lb4()[0], tile_fns_la4_lb4()[1]};
    return t;
}
const tile_fn *tile_table_la5()
{
    static const tile_fn t[] = {tile_fns_la5_lb0()[0], tile_fns_la5_lb0()[1], tile_fns_la5_lb1()[0], tile_fns_la5_lb1()[1], tile_fns_la5_lb2()[0], tile_fns_la5_lb2()[1], tile_fns_la5_lb3()[0], tile_fns_la5_lb3()[1]};
    return t;
}
const tile_fn *tile_table_la6()
{
    static const tile_fn t[] = {tile_fns_la6_lb0()[0], tile_fns_la6_lb0()[1], tile_fns_la6_lb1()[0], tile_fns_la6_lb1()[1], tile_fns_la6_lb2()[0], tile_fns_la6_lb2()[1], tile_fns_la6_lb3()[0], tile_fns_la6_lb3()[1]};
    return t;
}
const tile_fn *tile_table_la7()
{
    static const tile_fn t[] = {tile_fns_la7_lb0()[0], tile_fns_la7_lb0()[1], tile_fns_la7_lb1()[0], tile_fns_la7_lb1()[1], tile_fns_la7_lb2()[0], tile_fns_la7_lb2()[1], tile_fns_la7_lb3()[0], tile_fns_la7_lb3()[1]};
    return t;
}
const tile_fn *tile_table_la8()
{
    static const tile_fn t[] = {tile_fns_la8_lb0()[0], tile_fns_la8_lb0()[1], tile_fns_la8_lb1()[0], tile_fns_la8_lb1()[1], tile_fns_la8_lb2()[0], tile_fns_la8_lb2()[1], tile_fns_la8_lb3()[0], tile_fns_la8_lb3()[1]};
    return t;
}
const tile_fn *tile_table_la9()
{
    static const tile_fn t[] = {tile_fns_la9_lb0()[0], tile_fns_la9_lb0()[1], tile_fns_la9_lb1()[0], tile_fns_la9_lb1()[1], tile_fns_la9_lb2()[0], tile_fns_la9_lb2()[1], tile_fns_la9_lb3()[0], tile_fns_la9_lb3()[1]};
    return t;
}
}  // namespace shg
